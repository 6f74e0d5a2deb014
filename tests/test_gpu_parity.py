"""GPU parity: the HIP decoder against the oracle, element by element.

Every test goes through the C ABI (psb_decode_batch).  Tolerance: exact --
edge ids, weights and observable masks are integers."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import SEED, compare, compare_parallel, gpu_decode, say, valid_embedded

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1])
def test_d5_one_shot_config_all_shots(mode):
    """d=5, 5 rounds, p=q=0.005, 10,000 shots: every shot equals the oracle."""
    g = synth.rotated_phenom_graph(5, 0.005)
    s = synth.sample(g, 10000, seed=1)
    say(f"d5 mode={mode}: decoding 10000 shots")
    res = gpu_decode(g, s.syndromes, mode=mode)
    bad = compare(g, s.syndromes, res, range(10000))
    assert not bad, bad[:5]


def test_d11_batched_config_parity():
    """d=11, p=q=0.003: one persistent launch over 20,000 shots, all compared."""
    g = synth.rotated_phenom_graph(11, 0.003)
    s = synth.sample(g, 20000, seed=2)
    say("d11: decoding 20000 shots")
    res = gpu_decode(g, s.syndromes, levels=True)
    bad = compare(g, s.syndromes, res, range(20000))
    assert not bad, bad[:5]


@pytest.mark.parametrize("p,seed", [(0.005, 3), (0.001, 4)])
def test_d21_full_batch_sampled_parity(p, seed):
    """d=21 at the benchmark's launch shape (50,000 shots, default slots):
    150 sampled shots against the oracle, validity on every shot."""
    g = synth.rotated_phenom_graph(21, p)
    s = synth.sample(g, 50000, seed=seed)
    say(f"d21 p={p}: decoding 50000 shots")
    res = gpu_decode(g, s.syndromes)
    assert (res["status"] == 0).all(), np.bincount(res["status"])
    rng = np.random.default_rng(0)
    idx = sorted(set(rng.integers(0, 50000, 150).tolist()) | {0, 49999})
    bad = compare(g, s.syndromes, res, idx)
    assert not bad, bad[:5]
    assert not valid_embedded(g, s.syndromes, res)
    assert (res["weight"] <= s.weight).all()


def test_partition_equals_global_sparse_blossom():
    """Theorem 1: partition-and-fuse returns the same correction as global
    sparse blossom, on every shot of a d=21 batch."""
    g = synth.rotated_phenom_graph(21, 0.005)
    s = synth.sample(g, 20000, seed=5)
    a = gpu_decode(g, s.syndromes, mode=0)
    b = gpu_decode(g, s.syndromes, mode=1)
    for k in ("n_edges", "weight", "obs", "status"):
        assert np.array_equal(a[k], b[k]), k
    m = np.arange(a["edges"].shape[1])[None, :] < a["n_edges"][:, None]
    assert np.array_equal(np.where(m, a["edges"], 0), np.where(m, b["edges"], 0))


def test_high_error_rate_blossoms():
    """Dense syndromes (blossoms form and shatter) on d=11 and d=5."""
    for d, p, n in ((11, 0.03, 400), (5, 0.08, 2000)):
        g = synth.rotated_phenom_graph(d, p)
        s = synth.sample(g, n, seed=6)
        for mode in (0, 1):
            res = gpu_decode(g, s.syndromes, mode=mode)
            bad = compare(g, s.syndromes, res, range(n))
            assert not bad, (d, p, mode, bad[:5])


def test_random_and_repetition_graphs():
    for seed in range(3):
        g = synth.random_graph(60, 150, 10, 50, 90, seed, p=0.08)
        s = synth.sample(g, 300, seed=11)
        for mode, reading in ((0, 0), (1, 0), (0, 1)):
            res = gpu_decode(g, s.syndromes, mode=mode, reading=reading)
            bad = compare(g, s.syndromes, res, range(300))
            assert not bad, (seed, mode, reading, bad[:5])
    g = synth.repetition_graph(50, 100, 0.1)
    s = synth.sample(g, 500, seed=12)
    res = gpu_decode(g, s.syndromes)
    assert not compare(g, s.syndromes, res, range(500))
    g = synth.rotated_phenom_graph(9, 0.01, 0.03)      # unequal spatial / time weights
    s = synth.sample(g, 500, seed=13)
    res = gpu_decode(g, s.syndromes)
    assert not compare(g, s.syndromes, res, range(500))


@pytest.mark.parametrize("graph,walk", [("phenom", 0), ("circuit_uniform", 0), ("circuit_physical", 0),
                                        ("phenom_q02", 0), ("phenom", 1), ("circuit_uniform", 1),
                                        ("phenom_q02", 1)])
def test_cluster_levels_equal_oracle_clustering(graph, walk):
    """Processing-cluster levels (Methods, Algorithm "Clustering") against the
    oracle's plain construction: identical below the final level; at the
    final level every remaining event is placed there (the oracle may assign
    a later level to the same, single remaining component).  The level-1
    search enumerates paths of up to floor(b_1 / w_min) edges: 2 on the
    phenomenological and physical-noise graphs, 3 on the uniform-noise graph
    (its lightest edges are about 0.55 of the heaviest), 8 on a graph with
    timelike flips at q = 0.2.  The levels read the decoder's ball tables;
    walk = 1 makes them walk their paths (rows read in chunks, near lists from
    three edges on, the generic walk beyond three).  The final MWEM
    does not depend on the clusters (Theorem 1), so only this test checks
    them, and the results are compared with the oracle as well."""
    if graph == "phenom":
        g = synth.rotated_phenom_graph(11, 0.003)
    elif graph == "phenom_q02":
        g = synth.rotated_phenom_graph(11, 0.003, q=0.2)
    else:
        g = synth.rotated_circuit_graph(11, 0.003, graph.split("_")[1])
    s = synth.sample(g, 300, seed=14)
    res = gpu_decode(g, s.syndromes, levels=True, cluster_walk=walk)
    assert not compare(g, s.syndromes, res, range(0, 300, 3))
    og = oracle.Graph(g, SEED)
    import paper_2609_12262_amd as psb
    dec = psb.Decoder(psb.Graph.from_synth(g), tiebreak_seed=SEED)
    d_k, b_k, fin = dec.levels()
    kf = fin.index(1) + 1
    od, ob, _ = oracle.schedule(max(og.tiebroken_weights()), levels=max(len(d_k), 4))
    assert od[: len(d_k)] == d_k and ob[: len(b_k)] == b_k
    for i in range(300):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if len(dd) == 0:
            continue
        D, _ = og.defect_distances(dd)
        BT = og.boundary_table(dd)
        lv = oracle.cluster_levels(D, BT, od, ob)
        got = res["levels"][i, : len(dd)].tolist()
        for a, b in zip(got, lv):
            if b < kf:
                assert a == b, (i, got, lv)
            else:
                assert a == kf, (i, got, lv)


def test_edge_cases():
    g = synth.rotated_phenom_graph(5, 0.005)
    nb = g.nbytes
    # all-zero syndromes
    z = np.zeros((100, nb), np.uint8)
    res = gpu_decode(g, z)
    assert (res["status"] == 0).all() and (res["n_edges"] == 0).all() and (res["weight"] == 0).all()
    # single defects everywhere (ragged tail of the detector range)
    one = np.zeros((g.num_detectors, nb), np.uint8)
    for j in range(g.num_detectors):
        one[j, j >> 3] |= 1 << (j & 7)
    res = gpu_decode(g, one)
    assert not compare(g, one, res, range(g.num_detectors))
    # every detector active
    full = np.zeros((1, nb), np.uint8)
    for j in range(g.num_detectors):
        full[0, j >> 3] |= 1 << (j & 7)
    res = gpu_decode(g, full)
    assert not compare(g, full, res, [0])
    # truncated edge list: weight and obs still exact
    s = synth.sample(g, 500, seed=21)
    res = gpu_decode(g, s.syndromes, edges_per_shot=1)
    og = oracle.Graph(g, SEED)
    for i in range(500):
        r = og.mwem(synth.defects_of(s.syndromes[i], g.num_detectors))
        st = res["status"][i]
        assert st == (3 if len(r.edges) > 1 else 0)
        assert res["weight"][i] == r.weight and int(res["obs"][i]) == r.obs


def test_infeasible_component():
    # a triangle without boundary plus a path with a boundary edge
    g = synth.DetectorGraph(5, np.array([0, 1, 0, 3, 4], np.int32), np.array([1, 2, 2, 4, -1], np.int32),
                            np.array([3, 3, 3, 5, 5], np.int32), np.zeros(5, np.uint64), np.full(5, .1))
    rows = np.array([[0b00001], [0b00101], [0b01000], [0b11000]], np.uint8)
    res = gpu_decode(g, rows)
    assert res["status"].tolist()[0] == 2
    assert not compare(g, rows, res, range(4))


def test_determinism_and_order_independence():
    g = synth.rotated_phenom_graph(11, 0.01)
    s = synth.sample(g, 3000, seed=31)
    a = gpu_decode(g, s.syndromes)
    b = gpu_decode(g, s.syndromes)
    perm = np.random.default_rng(1).permutation(3000)
    c = gpu_decode(g, s.syndromes[perm])
    for k in ("n_edges", "weight", "obs", "status"):
        assert np.array_equal(a[k], b[k])
        assert np.array_equal(a[k][perm], c[k])


@pytest.mark.parametrize("fast_max_nodes,mode", [(24, 0), (24, 1), (-1, 0)])
def test_overflow_tier_parity(fast_max_nodes, mode):
    """Shots that exceed the fast tier's LDS capacities -- at intake or in the
    middle of the dynamics -- are finished by the overflow tier with the same
    result; fast_max_nodes = -1 runs every shot on that tier.  The overflow
    count equals the number of shots the oracle's explored set would not fit."""
    g = synth.rotated_phenom_graph(11, 0.01)
    s = synth.sample(g, 3000, seed=41)
    res = gpu_decode(g, s.syndromes, mode=mode, fast_max_nodes=fast_max_nodes, want_overflow=True)
    if fast_max_nodes > 0:
        assert 0 < res["n_overflow"] < 3000
    bad = compare(g, s.syndromes, res, range(3000))
    assert not bad, bad[:5]


def test_default_tiers_d21_overflow_share():
    """At the benchmark shape almost every shot stays in the fast tier."""
    g = synth.rotated_phenom_graph(21, 0.005)
    s = synth.sample(g, 20000, seed=42)
    res = gpu_decode(g, s.syndromes, want_overflow=True)
    assert (res["status"] == 0).all()
    assert res["n_overflow"] < 200
    rng = np.random.default_rng(3)
    assert not compare(g, s.syndromes, res, sorted(rng.integers(0, 20000, 60).tolist()))


def test_intake_rejected_by_both_tiers():
    """A shot with more detection events than max_defects_per_shot is rejected
    at intake by the fast tier and again by the overflow tier: status
    CAPACITY, empty outputs; the shots around it decode normally."""
    g = synth.rotated_phenom_graph(5, 0.005)
    nb = g.nbytes
    full = np.zeros((1, nb), np.uint8)
    for j in range(g.num_detectors):
        full[0, j >> 3] |= 1 << (j & 7)
    say("one shot, all detectors active, max_defects=8")
    res = gpu_decode(g, full, max_defects=8)
    assert res["status"].tolist() == [1]
    assert res["n_edges"][0] == 0 and res["weight"][0] == 0 and int(res["obs"][0]) == 0
    s = synth.sample(g, 400, seed=43)
    rows = np.concatenate([s.syndromes[:200], full, s.syndromes[200:]])
    say("401 shots with the full shot in the middle, max_defects=8")
    res = gpu_decode(g, rows, max_defects=8)
    counts = np.array([len(synth.defects_of(r, g.num_detectors)) for r in rows])
    assert (res["status"][counts > 8] == 1).all()
    keep = np.nonzero(counts <= 8)[0]
    assert not compare(g, rows, res, keep)


@pytest.mark.parametrize("fast_max_nodes,mode", [(0, 0), (0, 1), (24, 0)])
def test_lane_tier_parity(fast_max_nodes, mode):
    """The same engine with one shot per lane (first_tier = 1): every shot of
    a d=11 batch equals the oracle, including shots handed to the overflow
    tier."""
    g = synth.rotated_phenom_graph(11, 0.01)
    s = synth.sample(g, 3000, seed=44)
    say(f"lane tier d11 fast_max_nodes={fast_max_nodes} mode={mode}")
    res = gpu_decode(g, s.syndromes, mode=mode, fast_max_nodes=fast_max_nodes, first_tier=1, want_overflow=True)
    if fast_max_nodes > 0:
        assert 0 < res["n_overflow"] < 3000
    bad = compare(g, s.syndromes, res, range(3000))
    assert not bad, bad[:5]


def test_lane_tier_equals_wave_tier_d21():
    """At the benchmark shape the lane tier returns exactly the wavefront
    tier's outputs on every shot."""
    g = synth.rotated_phenom_graph(21, 0.005)
    s = synth.sample(g, 20000, seed=45)
    a = gpu_decode(g, s.syndromes, first_tier=0)
    b = gpu_decode(g, s.syndromes, first_tier=1)
    for k in ("n_edges", "weight", "obs", "status"):
        assert np.array_equal(a[k], b[k]), k
    m = np.arange(a["edges"].shape[1])[None, :] < a["n_edges"][:, None]
    assert np.array_equal(np.where(m, a["edges"], 0), np.where(m, b["edges"], 0))


def test_d11_config_100k_every_shot():
    """d=11, p=q=0.003: 100,000 shots in one persistent launch, every shot
    against the oracle."""
    g = synth.rotated_phenom_graph(11, 0.003)
    s = synth.sample(g, 100000, seed=2)
    say("d11: decoding 100000 shots")
    res = gpu_decode(g, s.syndromes)
    say("d11: comparing 100000 shots with the oracle")
    bad = compare_parallel(g, s.syndromes, res, range(100000))
    assert not bad, bad[:5]


def test_hash_map_large_graph_d41():
    """A graph above 32,768 detectors (d=41: 35,280) uses the per-shot hash
    instead of the direct detector map; shots of about 200 detection events
    go through both tiers."""
    g = synth.rotated_phenom_graph(41, 0.001)
    s = synth.sample(g, 32, seed=51)
    say("d41: decoding 32 shots")
    res = gpu_decode(g, s.syndromes, want_overflow=True)
    say(f"d41: {res['n_overflow']} shots on the overflow tier; comparing with the oracle")
    bad = compare_parallel(g, s.syndromes, res, range(32), chunk=2)
    assert not bad, bad[:5]


@pytest.mark.parametrize("first_tier,lds_state,caps", [(1, 0, (0, 0)), (0, 3, (1024, 768))])
def test_hash_map_large_graph_d41_other_first_tiers(first_tier, lds_state, caps):
    """The hash-map path (d=41) in the lane tier and in the wavefront tier with
    all state in LDS and large capacities: every shot equals the oracle."""
    g = synth.rotated_phenom_graph(41, 0.001)
    s = synth.sample(g, 32, seed=51)
    say(f"d41 first_tier={first_tier} lds_state={lds_state} caps={caps}: decoding 32 shots")
    res = gpu_decode(g, s.syndromes, first_tier=first_tier, fast_lds_state=lds_state, fast_max_nodes=caps[0],
                     fast_max_regions=caps[1])
    bad = compare_parallel(g, s.syndromes, res, range(32), chunk=2)
    assert not bad, bad[:5]


def test_server_windows_equal_oracle():
    """Serving: windows of three graphs, some with a uniform per-request
    weight, submitted one at a time in bursts (so several batches of one
    graph are in flight) and polled; every result equals the oracle on that
    window alone (with the request's weights)."""
    import time
    import paper_2609_12262_amd as psb
    gs = [synth.rotated_phenom_graph(d, 0.005) for d in (5, 9, 13)]
    Gs = [psb.Graph.from_synth(g) for g in gs]
    # per-graph options: default, wider first tier, one shot per lane
    srv = psb.Server(Gs, opts=[{}, {"fast_max_nodes": 640, "fast_max_regions": 416}, {"first_tier": 1}])
    rng = np.random.default_rng(61)
    reqs = []
    for j in range(600):
        k = int(rng.integers(0, 3))
        g = gs[k]
        row = synth.sample(g, 1, seed=1000 + j).syndromes[0]
        w = None
        if j % 3 == 0:
            p = float(rng.uniform(0.001, 0.007))
            w = np.full(g.num_edges, synth.weight_from_p(p), np.int32)
        reqs.append((k, row, w, srv.submit(k, row, w)))
        if j % 40 == 39:
            time.sleep(0.0003)   # batches overlap: later windows land on further in-flight batches
    say("server: 600 windows submitted")
    results = {}
    t0 = time.time()
    while len(results) < len(reqs) and time.time() - t0 < 60:
        for (k, row, w, t) in reqs:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
    srv.close()
    assert len(results) == len(reqs)
    oracles = {}
    for (k, row, w, t) in reqs:
        g = gs[k]
        if w is not None:
            g = synth.DetectorGraph(g.num_detectors, g.u, g.v, w, g.obs_mask, g.p)
        key = (k, None if w is None else int(w[0]))
        if key not in oracles:
            oracles[key] = oracle.Graph(g, SEED)
        ref = oracles[key].mwem(synth.defects_of(row, g.num_detectors))
        r = results[t]
        assert r["status"] == 0, (k, r)
        assert r["edges"].tolist() == ref.edges.tolist() and r["weight"] == ref.weight and r["obs"] == ref.obs
        assert r["latency_ns"] > 0


def test_server_budget_bursts_and_collect():
    """Serving under a device-memory budget: a budget too small for the
    decoders is refused with PSB_E_NOMEM; under one that fits, 2,000 windows
    of two graphs queued in bursts with per-window uniform weights
    (psb_server_submit_many) and collected in completion order
    (psb_server_collect) all equal the oracle with that window's weights, and
    the running statistics count every window."""
    import time
    import paper_2609_12262_amd as psb
    gs = [synth.rotated_phenom_graph(d, 0.005) for d in (7, 11)]
    Gs = [psb.Graph.from_synth(g) for g in gs]
    with pytest.raises(psb.PsbError, match="code -2"):
        psb.Server(Gs, opts={"num_slots": 256}, device_mem_budget=1 << 20)
    srv = psb.Server(Gs, opts={"num_slots": 256}, device_mem_budget=2 << 30)
    rng = np.random.default_rng(71)
    kinds, rows, wts, tickets = [], [], [], []
    for j0 in range(0, 2000, 250):
        kk = rng.integers(0, 2, 250)
        rr = [synth.sample(gs[k], 1, seed=9000 + j0 + i).syndromes[0] for i, k in enumerate(kk)]
        ww = [0 if (j0 + i) % 4 == 0 else synth.weight_from_p(float(rng.uniform(0.001, 0.007))) for i in range(250)]
        tickets += srv.submit_many(kk.tolist(), rr, ww)
        kinds += kk.tolist(); rows += rr; wts += ww
    say("server: 2000 windows queued in bursts")
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 60:
        for r in srv.collect():
            got[r["ticket"]] = r
    st = srv.stats()
    srv.close()
    assert len(got) == len(tickets)
    assert st["windows"] == len(tickets) and st["batches"] >= 1
    oracles = {}
    for idx in range(0, len(tickets), 5):
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


def test_server_cancel_and_wait():
    """Cancellation and time-outs in serving: of a 30,000-window burst, the
    last 200 are cancelled right after submission; every one still waiting
    completes at once with PSB_S_CANCELLED and is never decoded, any one
    already on the device completes normally.  psb_server_wait with a zero
    time-out returns at once; with a long one it returns when the window is
    done.  Every window that was not cancelled equals the oracle (sampled)."""
    import time
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(21, 0.005)
    G = psb.Graph.from_synth(g)
    srv = psb.Server([G])
    s = synth.sample(g, 30000, seed=77)
    rows = list(s.syndromes)
    tickets = srv.submit_many([0] * len(rows), rows)
    cancelled = {t for t in tickets[-200:] if srv.cancel(t)}
    say(f"server: {len(cancelled)} of the last 200 windows cancelled")
    assert cancelled, "the burst's tail should still be waiting"
    for t in list(cancelled)[:5]:
        assert srv.wait(t, 0)                     # already complete
    first_live = next(t for t in tickets if t not in cancelled)
    srv.wait(first_live, 0)                       # returns at once either way
    assert srv.wait(tickets[-201], 60_000_000)
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for r in srv.collect():
            got[r["ticket"]] = r
    srv.close(); G.close()
    assert len(got) == len(tickets)
    og = oracle.Graph(g, SEED)
    for i, t in enumerate(tickets):
        r = got[t]
        if t in cancelled:
            assert r["status"] == psb.PSB_S_CANCELLED and r["weight"] == 0
            continue
        assert r["status"] == 0, (i, r)
        if i % 97 == 0:
            ref = og.mwem(synth.defects_of(rows[i], g.num_detectors))
            assert r["weight"] == ref.weight and r["obs"] == ref.obs, i


@pytest.mark.parametrize("d,p,n,step", [(5, 0.003, 5000, 1), (9, 0.002, 3000, 1), (13, 0.002, 2000, 10)])
def test_circuit_x_graphs_equal_oracle(d, p, n, step):
    """Detector graphs from circuit-level X faults (diagonal spacetime edges,
    non-uniform weights, degree up to 10): shots equal the oracle."""
    g = synth.rotated_circuit_x_graph(d, p)
    s = synth.sample(g, n, seed=120 + d)
    say(f"circuit-x d={d}: decoding {n} shots")
    res = gpu_decode(g, s.syndromes)
    bad = compare(g, s.syndromes, res, range(0, n, step))
    assert not bad, bad[:5]


@pytest.mark.parametrize("model,d,p,n,step", [("uniform", 5, 0.003, 5000, 1), ("physical", 9, 0.003, 3000, 1),
                                              ("uniform", 13, 0.003, 2000, 10), ("physical", 21, 0.002, 2000, 20)])
def test_circuit_noise_model_graphs_equal_oracle(model, d, p, n, step):
    """X-memory detector graphs under the two circuit-level noise models
    (every fault of the syndrome-extraction circuit, degree up to 12, about
    twenty distinct weights): shots equal the oracle."""
    g = synth.rotated_circuit_graph(d, p, model)
    s = synth.sample(g, n, seed=150 + d)
    say(f"circuit {model} d={d} p={p}: decoding {n} shots")
    res = gpu_decode(g, s.syndromes)
    bad = compare(g, s.syndromes, res, range(0, n, step))
    assert not bad, bad[:5]


def test_circuit_uniform_d21_autotuned_graph_replay():
    """The benchmark's circuit-level workload (uniform noise, d=21, p=0.001,
    50,000 shots): the autotuned configuration, replayed through a captured
    HIP graph, equals the oracle on sampled shots and is valid on all."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_circuit_graph(21, 0.001, "uniform")
    s = synth.sample(g, 50000, seed=160)
    G = psb.Graph.from_synth(g)
    synd = torch.from_numpy(s.syndromes).cuda()
    say("circuit uniform d21: autotune")
    best, table = psb.autotune(G, synd[:8192], reps=1, tiebreak_seed=SEED)
    kw = {k: best[k] for k in ("fast_max_nodes", "fast_max_regions", "first_tier", "fast_lds_state")}
    say(f"circuit uniform d21: decoding 50000 shots with {kw}")
    res = gpu_decode(g, s.syndromes, **kw)
    G.close()
    assert (res["status"] == 0).all(), np.bincount(res["status"])
    assert not valid_embedded(g, s.syndromes, res)
    bad = compare_parallel(g, s.syndromes, res, range(0, 50000, 250))
    assert not bad, bad[:5]
