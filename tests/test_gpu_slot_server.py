"""GPU: slot-level serving (psb_slot_server), through the C ABI.  Every
window's result must equal the oracle's on that window alone, whatever was in
flight beside it.  No device-wide synchronisation while a server runs (its
persistent kernel would keep it waiting)."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import SEED, say

pytestmark = pytest.mark.gpu


def _collect_all(srv, n, limit_s=120):
    got = {}
    t0 = time.time()
    while len(got) < n and time.time() - t0 < limit_s:
        for r in srv.collect():
            got[r["ticket"]] = r
        time.sleep(0.001)
    return got


def test_slot_server_windows_equal_oracle_alone():
    """Three graphs (d=5, 9, 13), 3,000 windows in bursts of 250 with
    per-window uniform weights or the graph's own: more windows than the ring
    holds (so some wait on the host), and tight first-tier capacities on the
    d=13 group (so some windows take the overflow path).  Every window equals
    the oracle on that window alone."""
    import paper_2609_12262_amd as psb
    gs = [synth.rotated_phenom_graph(d, 0.006) for d in (5, 9, 13)]
    Gs = [psb.Graph.from_synth(g) for g in gs]
    opts = [{}, {}, {"fast_max_nodes": 28, "fast_max_regions": 28}]
    rng = np.random.default_rng(81)
    kinds, rows, wts = [], [], []
    for j0 in range(0, 3000, 250):
        kk = rng.integers(0, 3, 250)
        kinds += kk.tolist()
        rows += [synth.sample(gs[k], 1, seed=12000 + j0 + i).syndromes[0] for i, k in enumerate(kk)]
        wts += [0 if (j0 + i) % 3 == 0 else synth.weight_from_p(float(rng.uniform(0.001, 0.007))) for i in range(250)]
    srv = psb.SlotServer(Gs, opts=opts, waves=128, ring=512)
    try:
        tickets = []
        for j0 in range(0, 3000, 250):
            tickets += srv.submit_many(kinds[j0:j0 + 250], rows[j0:j0 + 250], wts[j0:j0 + 250])
        say("slot server: 3000 windows submitted")
        got = _collect_all(srv, len(tickets))
        st = srv.stats()
    finally:
        srv.close()
    for G in Gs:
        G.close()
    say(f"slot server stats: {st}")
    assert len(got) == len(tickets)
    assert st["windows"] == len(tickets) and st["overflow_redecoded"] > 0
    oracles = {}
    for idx in range(len(tickets)):
        k, row, w = kinds[idx], rows[idx], wts[idx]
        g = gs[k]
        if w:
            g = synth.DetectorGraph(g.num_detectors, g.u, g.v, np.full(g.num_edges, w, np.int32), g.obs_mask, g.p)
        key = (k, w)
        if key not in oracles:
            oracles[key] = oracle.Graph(g, SEED)
        ref = oracles[key].mwem(synth.defects_of(row, g.num_detectors))
        r = got[tickets[idx]]
        assert r["status"] == 0 and r["weight"] == ref.weight and r["obs"] == ref.obs, (idx, r, ref.weight, ref.obs)


def test_slot_server_edges_and_single_windows():
    """Edge lists through psb_slot_server_poll, on windows submitted one at a
    time with the slots idle in between (d=21, p=0.005): each equals the
    oracle's edge set."""
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(21, 0.005)
    G = psb.Graph.from_synth(g)
    s = synth.sample(g, 40, seed=83)
    og = oracle.Graph(g, SEED)
    got = []
    srv = psb.SlotServer([G], waves=64, ring=64)
    try:
        for i in range(40):
            t = srv.submit_many([0], [s.syndromes[i]])[0]
            r = None
            t0 = time.time()
            while r is None and time.time() - t0 < 30:
                r = srv.poll(t, edges_cap=2048)
            got.append(r)
            if r is None:
                break
    finally:
        srv.close()
    G.close()
    for i, r in enumerate(got):
        assert r is not None, i
        ref = og.mwem(synth.defects_of(s.syndromes[i], g.num_detectors))
        assert r["status"] == 0 and r["edges"].tolist() == ref.edges.tolist() and r["weight"] == ref.weight, i
