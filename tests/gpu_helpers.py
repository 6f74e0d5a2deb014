"""Helpers for GPU parity tests: run the HIP decoder through the C ABI and
compare with the oracle element by element."""
import sys

import numpy as np

import oracle
import synth

SEED = 0x5EED


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_decode(g, syndromes, mode=0, reading=0, max_defects=0, edges_per_shot=0, num_slots=0,
               levels=False, seed=SEED, timestamps=False, fast_max_nodes=0, fast_max_regions=0,
               overflow_slots=0, want_overflow=False, first_tier=0, fast_lds_state=0, cluster_walk=0):
    import torch
    import paper_2609_12262_amd as psb
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=seed, mode=mode, boundary_reading=reading, max_defects=max_defects,
                      edges_per_shot=edges_per_shot, num_slots=num_slots, fast_max_nodes=fast_max_nodes,
                      fast_max_regions=fast_max_regions, overflow_slots=overflow_slots, first_tier=first_tier,
                      fast_lds_state=fast_lds_state, cluster_walk=cluster_walk)
    synd = torch.from_numpy(np.ascontiguousarray(syndromes)).to("cuda")
    out = dec.decode(synd, levels=levels, timestamps=timestamps)
    torch.cuda.synchronize()
    res = dict(edges=out.edges.cpu().numpy(), n_edges=out.n_edges.cpu().numpy(),
               weight=out.weight.cpu().numpy(), obs=out.obs.cpu().numpy().view(np.uint64),
               status=out.status.cpu().numpy(),
               levels=out.levels.cpu().numpy() if levels else None,
               t_done=out.t_done.cpu().numpy() if timestamps else None)
    if want_overflow:
        res["n_overflow"] = dec.last_overflow()
    dec.close(); G.close()
    return res


def compare(g, syndromes, res, idx, seed=SEED, allow_status=()):
    """Indices (from idx) where the GPU result differs from the oracle."""
    og = oracle.Graph(g, seed)
    bad = []
    for i in idx:
        d = synth.defects_of(syndromes[i], g.num_detectors)
        r = og.mwem(d)
        st = int(res["status"][i])
        if r.flags & oracle.OF_INFEASIBLE:
            if st != 2:
                bad.append((i, "infeasible expected", st))
            continue
        if st in allow_status:
            continue
        got = res["edges"][i, : res["n_edges"][i]].tolist()
        if st != 0 or got != r.edges.tolist() or int(res["weight"][i]) != r.weight or int(res["obs"][i]) != r.obs:
            bad.append((i, st, len(d), int(res["weight"][i]), r.weight, int(res["obs"][i]), r.obs, r.flags))
    return bad


def valid_embedded(g, syndromes, res, chunk=2000):
    """Every returned edge set has odd degree exactly at the active detectors."""
    n = syndromes.shape[0]
    N = g.num_detectors
    bad = []
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        E = res["edges"][s0:s1]; NE = res["n_edges"][s0:s1]
        mask = np.arange(E.shape[1])[None, :] < NE[:, None]
        rows = np.repeat(np.arange(s1 - s0), mask.sum(1))
        ee = E[mask]
        par = np.zeros((s1 - s0) * N + 1, np.int64)
        for ends in (g.u[ee], g.v[ee]):
            ok = ends >= 0
            np.add.at(par, rows[ok] * N + ends[ok], 1)
        par = (par[:-1] % 2).reshape(s1 - s0, N).astype(np.uint8)
        want = np.unpackbits(syndromes[s0:s1], axis=1, bitorder="little")[:, :N]
        diff = np.nonzero((par != want).any(1))[0]
        bad.extend((s0 + diff).tolist())
    return bad


_PAR = None


def _par_init(g, seed, syndromes, res):
    global _PAR
    _PAR = (g, seed, syndromes, res)


def _par_chunk(idx):
    g, seed, syndromes, res = _PAR
    return compare(g, syndromes, res, idx, seed)


def compare_parallel(g, syndromes, res, idx, seed=SEED, workers=16, chunk=64):
    """compare() spread over host processes (forked; the children only run the CPU oracle)."""
    import multiprocessing as mp
    idx = list(idx)
    parts = [idx[i:i + chunk] for i in range(0, len(idx), chunk)]
    ctx = mp.get_context("fork")
    keep = {k: res[k] for k in ("edges", "n_edges", "weight", "obs", "status")}
    with ctx.Pool(min(workers, len(parts)), initializer=_par_init, initargs=(g, seed, syndromes, keep)) as pool:
        bad = []
        for b in pool.imap(_par_chunk, parts):
            bad.extend(b)
    return bad


_SB = None


def _sb_init(g, seed, syndromes, res):
    global _SB
    _SB = (g, oracle.SparseBlossom(g, seed), syndromes, res)


def _sb_chunk(idx):
    g, sb, syndromes, res = _SB
    bad = []
    for i in idx:
        r = sb.decode(synth.defects_of(syndromes[i], g.num_detectors), global_mode=True)
        st = int(res["status"][i])
        if r.flags & oracle.SBF_INFEASIBLE:
            if st != 2:
                bad.append((i, "infeasible expected", st))
            continue
        got = res["edges"][i, : res["n_edges"][i]].tolist()
        if r.flags or st != 0 or got != r.edges.tolist() or int(res["weight"][i]) != r.weight or int(res["obs"][i]) != r.obs:
            bad.append((i, st, int(res["weight"][i]), r.weight, int(res["obs"][i]), r.obs, r.flags))
    return bad


def compare_sb_parallel(g, syndromes, res, idx, seed=SEED, workers=16, chunk=500):
    """Every shot in idx against the serial sparse-blossom oracle (global mode; pinned to the Dijkstra +
    Edmonds MWEM on every shot of the small configurations and on samples of the large ones), spread over
    host processes."""
    import multiprocessing as mp
    idx = list(idx)
    parts = [idx[i:i + chunk] for i in range(0, len(idx), chunk)]
    keep = {k: res[k] for k in ("edges", "n_edges", "weight", "obs", "status")}
    with mp.get_context("fork").Pool(min(workers, len(parts)), initializer=_sb_init,
                                     initargs=(g, seed, syndromes, keep)) as pool:
        bad = []
        for b in pool.imap(_sb_chunk, parts):
            bad.extend(b)
    return bad
