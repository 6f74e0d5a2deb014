"""Pins for the oracle: results fixed by the paper's definitions, closed forms,
brute force and textbook routines -- never by re-running the oracle itself."""
import itertools
import os
from collections import deque
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

SEED = 0x5EED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- tie-break
def test_splitmix_matches_published_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_outputs.txt")) if l.strip() and l[0] != "#"]
    for seed, k, out in rows:
        assert oracle.splitmix_output(int(seed), int(k)) == int(out)


def test_c_tiebreak_equals_definition():
    g = synth.rotated_phenom_graph(5, 0.005)
    og = oracle.Graph(g, SEED)
    got = og.tiebroken_weights()
    for e in range(g.num_edges):
        h = oracle.splitmix_output(SEED, e + 1) >> 24
        assert got[e] == (2 * int(g.w[e]) << 64) + 2 * h
        assert got[e] % 2 == 0                      # even weights (Supplementary S1)
    # sum of all secondary parts stays below one primary unit
    assert sum(x & ((1 << 64) - 1) for x in got) < (1 << 64)


# ---------------------------------------------------------------- distances
def _bfs_hops(g, src):
    adj = [[] for _ in range(g.num_detectors)]
    bd = [False] * g.num_detectors
    for a, b in zip(g.u.tolist(), g.v.tolist()):
        if b < 0:
            bd[a] = True
        else:
            adj[a].append(b); adj[b].append(a)
    dist = [-1] * g.num_detectors
    dist[src] = 0
    q = deque([src])
    while q:
        x = q.popleft()
        for y in adj[x]:
            if dist[y] < 0:
                dist[y] = dist[x] + 1; q.append(y)
    bdh = min(dist[x] + 1 for x in range(g.num_detectors) if bd[x] and dist[x] >= 0)
    return dist, bdh


@pytest.mark.parametrize("d", [5, 7])
def test_dijkstra_primary_equals_bfs_hops(d):
    """Uniform weights: primary distance = 2w * hop count (textbook BFS)."""
    g = synth.rotated_phenom_graph(d, 0.01)
    og = oracle.Graph(g, SEED)
    w2 = 2 * int(g.w[0])
    for src in (0, g.num_detectors // 2, g.num_detectors - 1):
        dist, _, bd, _ = og.dijkstra(src)
        hops, bdh = _bfs_hops(g, src)
        for x in range(g.num_detectors):
            assert dist[x] >> 64 == w2 * hops[x]
        assert bd >> 64 == w2 * bdh


# ---------------------------------------------------------------- matching
def _brute_max_weight_matching(W):
    n = len(W)
    best = 0

    def rec(free, acc):
        nonlocal best
        best = max(best, acc)
        if len(free) < 2:
            return
        i = free[0]
        rec(free[1:], acc)                      # i unmatched
        for j in free[1:]:
            if W[i][j] > 0:
                rec([x for x in free[1:] if x != j], acc + W[i][j])

    rec(list(range(n)), 0)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_edmonds_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 10))
    W = [[0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < 0.7:
                # large, tie-prone values exercise the 128-bit arithmetic
                W[i][j] = W[j][i] = int(rng.integers(1, 6)) * (1 << 70) + int(rng.integers(0, 3))
    mate, ok = oracle.max_weight_matching(W)
    assert ok, "LP certificate failed"
    got = sum(W[i][mate[i]] for i in range(n) if mate[i] > i)
    assert got == _brute_max_weight_matching(W)
    for i in range(n):
        if mate[i] >= 0:
            assert mate[mate[i]] == i and W[i][mate[i]] > 0


def test_edmonds_matches_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(7)
    for trial in range(6):
        n = 30
        W = [[0] * n for _ in range(n)]
        G = nx.Graph()
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < 0.3:
                    x = int(rng.integers(1, 50))
                    W[i][j] = W[j][i] = x
                    G.add_edge(i, j, weight=x)
        mate, ok = oracle.max_weight_matching(W)
        assert ok
        ref = nx.max_weight_matching(G)
        assert sum(W[i][mate[i]] for i in range(n) if mate[i] > i) == sum(W[a][b] for a, b in ref)


# ---------------------------------------------------------------- MWEM
def _check_valid_embedded_matching(g, defects, edges):
    deg = np.zeros(g.num_detectors, np.int64)
    for e in edges:
        deg[g.u[e]] ^= 1
        if g.v[e] >= 0:
            deg[g.v[e]] ^= 1
    assert set(np.nonzero(deg)[0].tolist()) == set(int(x) for x in defects)


@pytest.mark.parametrize("n_det", [1, 3, 6, 10])
def test_mwem_repetition_equals_edge_subset_brute_force(n_det):
    rng = np.random.default_rng(n_det)
    w = rng.integers(3, 9, n_det + 1)
    g = synth.repetition_graph(n_det, w)
    og = oracle.Graph(g, SEED)
    for mask in range(1 << n_det):
        defects = [i for i in range(n_det) if mask >> i & 1]
        r = og.mwem(defects)
        assert r.flags & (oracle.OF_CERT_FAIL | oracle.OF_INFEASIBLE) == 0
        ref = oracle.brute_mwem_edges(g, defects, SEED)
        assert r.edges.tolist() == ref
        assert r.weight == int(sum(int(g.w[e]) for e in ref))


def _repetition_dp(w, defects, n_det):
    """Linear DP on the path graph: edge i is used iff the parity of defects
    left of it is odd (a T-join on a path with a free boundary at both ends
    is fixed by the choice of the first edge)."""
    best = None
    for first in (0, 1):
        used = [first]
        par = first
        for i in range(n_det):
            par ^= (1 if i in defects else 0)
            used.append(par)
        # the last edge goes to the right boundary, any parity allowed
        tot = sum(int(w[i]) for i in range(n_det + 1) if used[i])
        best = tot if best is None else min(best, tot)
    return best


def test_mwem_repetition_weight_equals_dp():
    rng = np.random.default_rng(3)
    n_det = 40
    w = rng.integers(1, 20, n_det + 1)
    g = synth.repetition_graph(n_det, w)
    og = oracle.Graph(g, SEED)
    for _ in range(50):
        defects = sorted(set(rng.integers(0, n_det, int(rng.integers(0, 12))).tolist()))
        r = og.mwem(defects)
        assert r.weight == _repetition_dp(w, set(defects), n_det)
        _check_valid_embedded_matching(g, defects, r.edges)


@pytest.mark.parametrize("seed", range(8))
def test_mwem_random_graph_equals_edge_subset_brute_force(seed):
    g = synth.random_graph(n_det=9, n_edges=20, n_boundary=3, wmin=1, wmax=4, seed=seed)
    og = oracle.Graph(g, SEED)
    rng = np.random.default_rng(100 + seed)
    for _ in range(12):
        defects = sorted(set(rng.integers(0, 9, int(rng.integers(0, 7))).tolist()))
        r = og.mwem(defects)
        ref = oracle.brute_mwem_edges(g, defects, SEED)
        assert ref is not None
        assert r.edges.tolist() == ref
        assert r.obs == int(np.bitwise_xor.reduce(g.obs_mask[ref])) if ref else r.obs == 0


def test_mwem_pairing_cost_equals_brute_force_pairing():
    """<= 10 defects: the matched cost equals the exhaustive minimum over all
    pairings (defect-defect or defect-boundary) of the exact distances."""
    g = synth.rotated_phenom_graph(5, 0.02)
    og = oracle.Graph(g, SEED)
    s = synth.sample(g, 300, seed=11)
    wt = og.tiebroken_weights()
    checked = 0
    for i in range(300):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if not (1 <= len(dd) <= 10):
            continue
        D, BD = og.defect_distances(dd)
        ref = oracle.brute_min_pairing(D, BD)
        r = og.mwem(dd)
        assert sum(wt[e] for e in r.edges) == ref
        checked += 1
    assert checked > 50


def test_mwem_closed_form_cases():
    g = synth.rotated_phenom_graph(5, 0.005)
    og = oracle.Graph(g, SEED)
    wt = og.tiebroken_weights()
    # isolated adjacent pair: M = that edge
    e = int(np.nonzero((g.v >= 0))[0][len(g.v) // 3])
    a, b = int(g.u[e]), int(g.v[e])
    r = og.mwem(sorted([a, b]))
    assert r.edges.tolist() == [e] and r.weight == int(g.w[e])
    # single defect on a boundary edge: M = its cheapest boundary edge
    eb = int(np.nonzero(g.v < 0)[0][0])
    u = int(g.u[eb])
    cands = [x for x in range(g.num_edges) if g.v[x] < 0 and g.u[x] == u]
    r = og.mwem([u])
    assert r.edges.tolist() == [min(cands, key=lambda x: wt[x])]
    # empty syndrome
    r = og.mwem([])
    assert r.edges.size == 0 and r.weight == 0 and r.obs == 0 and r.flags == 0


@pytest.mark.parametrize("d,p,n", [(5, 0.005, 400), (11, 0.003, 60)])
def test_mwem_certificate_validity_and_bound(d, p, n):
    """LP certificate holds, output is a valid embedded matching, and its
    weight never exceeds the sampled error's weight (N is feasible)."""
    g = synth.rotated_phenom_graph(d, p)
    og = oracle.Graph(g, SEED)
    s = synth.sample(g, n, seed=2)
    for i in range(n):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        r = og.mwem(dd)
        assert r.flags & (oracle.OF_CERT_FAIL | oracle.OF_INFEASIBLE | oracle.OF_CAPACITY) == 0
        _check_valid_embedded_matching(g, dd, r.edges)
        assert r.weight <= s.weight[i]


def test_infeasible_without_boundary():
    # a triangle with no boundary edge: one defect cannot be matched
    g = synth.DetectorGraph(3, np.array([0, 1, 0], np.int32), np.array([1, 2, 2], np.int32),
                            np.array([1, 1, 1], np.int32), np.zeros(3, np.uint64), np.full(3, .1))
    og = oracle.Graph(g, SEED)
    assert og.mwem([0]).flags & oracle.OF_INFEASIBLE
    assert og.mwem([0, 2]).flags == 0


# ---------------------------------------------------------------- schedule
@pytest.mark.parametrize("w", [2710, 2972, 3536, 2536, 10, 1])
def test_schedule_closed_form_first_levels(w):
    """Hand derivation for q = 1/10, phi_min = 1/100: with phi_1 = 1 the binding
    condition is 1 > 2 d_1 / b, so b_1 = 2 d_1 + 1 (the Phi condition needs
    only b >= (3/0.891 - 2) d_1); then d_2 = 3 d_1 + 4 b_1 + 2 w = 13 w + 15."""
    d, b, phi = oracle.schedule(w, levels=3)
    assert d[0] == w + 1
    assert b[0] == 2 * d[0] + 1
    assert d[1] == 13 * w + 15
    assert phi[1] == 1 - Fraction(3 * d[0], 2 * d[0] + b[0])


@pytest.mark.parametrize("w", [2710, 3536, 7])
def test_schedule_properties(w):
    """Supplementary S11: phi_k >= phi_bar_k, every b_k admissible and minimal,
    b_k >= d_k, d_{k+1} = 3 d_k + 4 b_k + 2 w_max."""
    q, pm = Fraction(1, 10), Fraction(1, 100)
    d, b, phi = oracle.schedule(w, q, pm, levels=5)
    for k in range(5):
        assert phi[k] >= oracle.phi_bar(k + 1, q, pm)
        tgt = oracle.phi_bar(k + 2, q, pm)
        assert b[k] >= d[k] and phi[k] > Fraction(2 * d[k], b[k])
        assert oracle.Phi_next(b[k], d[k], phi[k]) >= tgt
        bm = b[k] - 1
        assert not (bm >= d[k] and phi[k] > Fraction(2 * d[k], bm) and oracle.Phi_next(bm, d[k], phi[k]) >= tgt)
        if k + 1 < 5:
            assert d[k + 1] == 3 * d[k] + 4 * b[k] + 2 * w


# ---------------------------------------------------------------- clustering
def _cluster_case(defects, g, reading="strict"):
    og = oracle.Graph(g, SEED)
    D, _ = og.defect_distances(defects)
    BT = og.boundary_table(defects)
    wmax = max(og.tiebroken_weights())
    d, b, _ = oracle.schedule(wmax, levels=4)
    return oracle.cluster_levels(D, BT, d, b, reading), D, d, b


def test_clustering_isolated_pair_and_boundary_single():
    g = synth.rotated_phenom_graph(11, 0.003)
    # pick an interior spatial edge in layer 6 and a boundary detector in layer 2
    nz = (11 * 11 - 1) // 2
    e = next(x for x in range(g.num_edges) if g.v[x] >= 0 and g.u[x] // nz == 5 and g.u[x] % nz > 20)
    a, b = int(g.u[e]), int(g.v[e])
    eb = next(x for x in range(g.num_edges) if g.v[x] < 0 and g.u[x] // nz == 1)
    c = int(g.u[eb])
    defects = sorted([a, b, c])
    lv, _, _, _ = _cluster_case(defects, g)
    assert lv == [1, 1, 1]


def test_clustering_chain_of_three_not_level_one():
    """Three defects two hops apart in a row: linked at level 1 (<= b_1) but
    diameter > d_1, so none is level 1; with even... (odd, no boundary within
    d_2) they stay together at a higher level."""
    g = synth.rotated_phenom_graph(11, 0.003)
    nz = (11 * 11 - 1) // 2
    base = 5 * nz
    # timelike chain: same face in layers 4, 6, 8 (two timelike hops apart)
    f = 30
    defects = [3 * nz + f, 5 * nz + f, 7 * nz + f]
    lv, D, d, b = _cluster_case(defects, g)
    assert D[0][1] <= b[0] and D[0][2] > d[0]
    assert lv[0] == lv[1] == lv[2] and lv[0] >= 2


def test_clustering_partition_properties():
    """Every accepted cluster: diameter <= d_k, separation > b_k from the
    residual of its level, parity condition (Methods, Definition of the
    processing-cluster hierarchy; Supplementary S2 cluster condition)."""
    g = synth.rotated_phenom_graph(11, 0.01)
    og = oracle.Graph(g, SEED)
    wmax = max(og.tiebroken_weights())
    d, b, _ = oracle.schedule(wmax, levels=4)
    s = synth.sample(g, 40, seed=5)
    for i in range(40):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if len(dd) == 0:
            continue
        D, _ = og.defect_distances(dd)
        BT = og.boundary_table(dd)
        lv = oracle.cluster_levels(D, BT, d, b)
        m = len(dd)
        for k in sorted(set(lv)):
            if k == 0:
                continue
            resid = [x for x in range(m) if lv[x] >= k or lv[x] == 0]
            members = [x for x in range(m) if lv[x] == k]
            for x in members:
                for y in members:
                    pass
            # separation of level-k defects from level > k residual
            for x in members:
                for y in resid:
                    if lv[y] != k:
                        assert D[x][y] is None or D[x][y] > b[k - 1]


# ---------------------------------------------------------------------------
# Sliding-window decoding (oracle.window_schedule / window_decode)
# ---------------------------------------------------------------------------

def _window_setup(d, rounds, W, C, p, n, seed):
    g = synth.rotated_phenom_graph(d, p, rounds=rounds)
    L = (d * d - 1) // 2
    sch = oracle.window_schedule(g, L, W, C)
    gs = [oracle.Graph(wg, 0x5EED) for _, wg, _, _ in sch]
    s = synth.sample(g, n, seed=seed)
    return g, L, sch, gs, s


def test_window_schedule_structure():
    """Windows start every C layers; all but the last have W layers; the last
    reaches the final layer; every window edge maps to a full-graph edge with
    an end in the window, and the last window commits everything."""
    g, L, sch, _, _ = _window_setup(5, 12, 6, 3, 0.01, 1, 1)
    n_layers = g.num_detectors // L
    assert [a for a, *_ in sch] == [0, 3, 6, 9]
    for k, (a, wg, emap, commit) in enumerate(sch):
        last = k == len(sch) - 1
        assert wg.num_detectors == L * ((n_layers - a) if last else 6)
        assert len(emap) == wg.num_edges == len(commit)
        if last:
            assert all(commit)
        for e, ge in enumerate(emap):
            ends = [x for x in (int(g.u[ge]), int(g.v[ge])) if x >= 0]
            assert any(a * L <= x < a * L + wg.num_detectors for x in ends)


def test_window_single_window_equals_mwem():
    """A window covering every layer is the whole graph: the MWEM itself."""
    g, L, sch, gs, s = _window_setup(5, 8, 100, 3, 0.01, 60, 2)
    assert len(sch) == 1
    full = oracle.Graph(g, 0x5EED)
    for i in range(60):
        d = synth.defects_of(s.syndromes[i], g.num_detectors)
        r = full.mwem(d)
        w, o, ok = oracle.window_decode(g, sch, gs, L, d)
        assert ok and (w, o) == (r.weight, r.obs)


def test_window_decode_is_a_valid_correction():
    """Committed edges resolve every detection event (the running syndrome
    ends empty) and weigh at least the MWEM."""
    g, L, sch, gs, s = _window_setup(5, 16, 6, 2, 0.02, 80, 3)
    full = oracle.Graph(g, 0x5EED)
    for i in range(80):
        d = synth.defects_of(s.syndromes[i], g.num_detectors)
        w, o, ok = oracle.window_decode(g, sch, gs, L, d)
        assert ok and w >= full.mwem(d).weight


# ---------------------------------------------------------------------------
# Complementary gap (oracle.Complementary)
# ---------------------------------------------------------------------------

def _brute_constrained(g, defects, bit=1):
    """Minimum weight over all edge subsets with odd degree exactly at the
    defects, split by the observable bit (tiny graphs)."""
    best = [None, None]
    E = g.num_edges
    want = set(int(x) for x in defects)
    for mask in range(1 << E):
        deg = {}
        wsum, ob = 0, 0
        for e in range(E):
            if mask >> e & 1:
                wsum += int(g.w[e]); ob ^= int(g.obs_mask[e])
                for x in (int(g.u[e]), int(g.v[e])):
                    if x >= 0:
                        deg[x] = deg.get(x, 0) ^ 1
        if {x for x, k in deg.items() if k} != want:
            continue
        b = 1 if ob & bit else 0
        if best[b] is None or wsum < best[b]:
            best[b] = wsum
    return tuple(best)


def test_complementary_equals_brute_force_on_small_graphs():
    """Both constrained minima equal brute force over every edge subset: a
    repetition code with uneven weights (observable on the left boundary) and
    a d=3 rotated code over one round (observable on the top boundary)."""
    rng = np.random.default_rng(5)
    rep = synth.repetition_graph(7, rng.integers(1, 9, 8).tolist())
    rot = synth.rotated_phenom_graph(3, 0.01, rounds=1)
    assert rot.num_edges <= 16
    for g in (rep, rot):
        co = oracle.Complementary(g, 0, 0x5EED)
        for t in range(12):
            k = int(rng.integers(0, min(5, g.num_detectors) + 1))
            defects = sorted(rng.choice(g.num_detectors, size=k, replace=False).tolist())
            assert co.weights(defects) == _brute_constrained(g, defects), (g.num_detectors, defects)


def test_complementary_minimum_is_the_mwem():
    """The lighter constrained minimum is the MWEM weight, on the side of the
    MWEM's observable bit."""
    g = synth.rotated_phenom_graph(5, 0.02)
    co = oracle.Complementary(g, 0, 0x5EED)
    og = oracle.Graph(g, 0x5EED)
    s = synth.sample(g, 80, seed=6)
    for i in range(80):
        d = synth.defects_of(s.syndromes[i], g.num_detectors)
        w0, w1 = co.weights(d)
        r = og.mwem(d)
        assert min(w0, w1) == r.weight
        if w0 != w1:
            assert (w1 < w0) == bool(r.obs & 1)
