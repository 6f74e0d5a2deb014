"""The allocation-free entry point psb_decode_batch_noalloc against
psb_decode_batch, through the C ABI: two calls in a row on one decoder, the
second with a smaller batch, every output equal element by element; the first
call sends shots through the overflow list that lives in the library's fixed
device array.  A batch above the limit is refused before anything runs."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import SEED, compare, say

pytestmark = pytest.mark.gpu

KEYS = ("n_edges", "weight", "obs", "status")


def _host(out):
    h = {k: getattr(out, k).cpu().numpy() for k in KEYS}
    e = out.edges.cpu().numpy()
    h["edges"] = np.where(np.arange(e.shape[1])[None, :] < h["n_edges"][:, None], e, -1)
    return h


def test_noalloc_equals_decode_batch_on_two_calls():
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(21, 0.005)
    G = psb.Graph.from_synth(g)
    # a small first tier, so that part of every batch goes through the overflow list
    dec = psb.Decoder(G, tiebreak_seed=SEED, fast_max_nodes=150, fast_max_regions=150)
    for n, seed in ((3000, 41), (700, 42)):
        syn = synth.sample(g, n, seed=seed).syndromes
        S = torch.from_numpy(syn).cuda()
        say(f"noalloc: {n} shots")
        want = dec.decode(S)
        torch.cuda.synchronize()
        ovf_ref = dec.last_overflow()
        want = _host(want)
        got = dec.alloc(n)
        got.edges.fill_(-7); got.n_edges.fill_(-7); got.status.fill_(-7)
        dec.decode_into_noalloc(S, got)
        torch.cuda.synchronize()
        ovf = dec.last_overflow()
        got = _host(got)
        for key in ("edges",) + KEYS:
            assert np.array_equal(got[key], want[key]), (n, key)
        assert ovf == ovf_ref and ovf > 0, (ovf, ovf_ref)
        res = dict(got, obs=got["obs"].view(np.uint64))
        bad = compare(g, syn, res, range(0, n, 25))
        assert not bad, bad[:5]
        say(f"noalloc: {n} shots equal, {ovf} through the overflow list")
    # beyond the limit: refused on the host, nothing launched
    one = torch.zeros(8, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(one.data_ptr())
    big = psb.lib().psb_decode_batch_noalloc(dec._h, p, ctypes.c_int64((1 << 20) + 1), p, p, p, p, p,
                                             ctypes.c_void_p(0), ctypes.c_void_p(0), ctypes.c_void_p(0),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert big == psb.PSB_E_INVALID if hasattr(psb, "PSB_E_INVALID") else big == -1
    torch.cuda.synchronize()
    dec.close(); G.close()
