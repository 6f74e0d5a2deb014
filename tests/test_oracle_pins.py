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
    processing-cluster hierarchy; Supplementary S2 cluster condition).  The
    checks are made on the exact distance tables, independently of how
    cluster_levels builds its components."""
    g = synth.rotated_phenom_graph(11, 0.01)
    og = oracle.Graph(g, SEED)
    wmax = max(og.tiebroken_weights())
    d, b, _ = oracle.schedule(wmax, levels=4)
    s = synth.sample(g, 40, seed=5)
    n_odd = n_multi = 0
    for i in range(40):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if len(dd) == 0:
            continue
        D, _ = og.defect_distances(dd)
        BT = og.boundary_table(dd)
        lv, comps = oracle.cluster_levels(D, BT, d, b, components=True)
        m = len(dd)
        assert all(x > 0 for x in lv)
        assert sorted(x for _, c in comps for x in c) == list(range(m))     # a partition of the events
        for k, members in comps:
            assert all(lv[x] == k for x in members)
            # diameter of the event set
            for x in members:
                for y in members:
                    assert D[x][y] is not None and D[x][y] <= d[k - 1]
            # parity: even, or (strict reading) one boundary vertex within d_k of every member
            if len(members) % 2 == 1:
                n_odd += 1
                assert any(all(BT[x][j] is not None and BT[x][j] <= d[k - 1] for x in members)
                           for j in range(len(BT[members[0]])))
            n_multi += len(members) > 1
            # separation from every event still residual at level k that is not in this cluster
            for x in members:
                for y in range(m):
                    if y not in members and lv[y] >= k:
                        assert D[x][y] is None or D[x][y] > b[k - 1]
    assert n_odd > 0 and n_multi > 0


def test_clustering_loose_and_strict_readings_differ_on_an_odd_cluster():
    """A hand-built odd cluster: three events on a 60-detector path (weights
    10, doubled 20), two adjacent (29, 30) and one two edges away (32).  All
    three are linked at level 1 (29-30 one edge, 30-32 two edges: 40 plus
    tie-break parts, within b_1 = 2 d_1 + 1 with d_1 = w_max + 1) but the
    diameter (29 to 32, 60) exceeds d_1
    (about 20), so they stay residual; at level 2 the exploring regions cover
    the path, the diameter fits d_2 = 3 d_1 + 4 b_1 + 2 w_max (about 260) and
    the set is odd.  Its nearest boundary vertex is 28 edges (560) from detector 32 and
    30 edges from detector 29: beyond d_2, so the strict reading (one boundary
    vertex within d_k of every member) rejects it until level 3, while the
    loose reading (some member's exploring region of radius b_2/2 reaches a
    boundary vertex) accepts it at level 2."""
    g = synth.repetition_graph(60, 10)
    defects = [29, 30, 32]
    og = oracle.Graph(g, SEED)
    d, b, _ = oracle.schedule(max(og.tiebroken_weights()), levels=4)
    D, _ = og.defect_distances(defects)
    BT = og.boundary_table(defects)
    assert max(D[0][1], D[0][2], D[1][2]) >> 64 == 60 and d[0] >> 64 == 20 and D[1][2] <= b[0] and D[0][2] > d[0]
    assert min(min(x for x in row) for row in BT) >> 64 == 560 and min(BT[2]) > d[1]
    assert oracle.cluster_levels(D, BT, d, b, "strict") == [3, 3, 3]
    assert oracle.cluster_levels(D, BT, d, b, "loose") == [2, 2, 2]


def test_schedule_level_two_and_three_closed_forms():
    """Levels 2 and 3 of the schedule (Methods, Algorithm "Parameter schedule";
    q = 1/10, phi_min = 1/100) at w_max = 2710, 2972, 3536 and 2536 (the
    benchmark weights doubled), derived here from the algorithm's inequalities
    solved for b in closed form:
      phi_2 = Phi_2(b_1) = 1 - 3 d_1 / (2 d_1 + b_1)            (phi_1 = 1),
      Phi_3(b) >= phi_bar_3  <=>  b >= ((phi_2 + 2) d_2 / (phi_2 - phi_bar_3) - (phi_2 + 1) d_2) / phi_2,
    and b_2 also exceeds 2 d_2 / phi_2; d_{k+1} = 3 d_k + 4 b_k + 2 w_max."""
    import math
    q, pm = Fraction(1, 10), Fraction(1, 100)
    expect = {2710: (35245, 1201614, 4917611), 2972: (38651, 1317805, 5393117),
              3536: (45983, 1567924, 6416717), 2536: (32983, 1124450, 4601821)}
    for w, (d2_e, b2_e, d3_e) in expect.items():
        d1 = w + 1
        b1 = 2 * d1 + 1
        phi2 = 1 - Fraction(3 * d1, 2 * d1 + b1)
        d2 = 3 * d1 + 4 * b1 + 2 * w
        target3 = pm + (1 - pm) * q ** 2
        lo = ((phi2 + 2) * d2 / (phi2 - target3) - (phi2 + 1) * d2) / phi2
        b2 = max(d2, math.floor(2 * d2 / phi2) + 1, math.ceil(lo))
        d3 = 3 * d2 + 4 * b2 + 2 * w
        assert (d2, b2, d3) == (d2_e, b2_e, d3_e)
        od, ob, ophi = oracle.schedule(w, q, pm, levels=3)
        assert (od[1], ob[1], od[2]) == (d2, b2, d3)
        assert ophi[1] == phi2 and abs(float(ophi[1]) - 0.2500) < 1e-3 and abs(float(ophi[2]) - 0.0199) < 1e-4


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


def _parity_search(g, bit, starts):
    """Dijkstra over (detector, observable parity) states with the caller's
    weights; `starts` = [(detector, parity, distance)].  Returns the distance
    to every (detector, parity) and to every (boundary edge, parity) end."""
    import heapq
    adj = [[] for _ in range(g.num_detectors)]
    for e in range(g.num_edges):
        a, b = int(g.u[e]), int(g.v[e])
        adj[a].append((e, b))
        if b >= 0:
            adj[b].append((e, a))
    dist = {}
    bd = {}
    h = [(dd, x, par) for x, par, dd in starts]
    heapq.heapify(h)
    while h:
        dd, x, par = heapq.heappop(h)
        if (x, par) in dist:
            continue
        dist[(x, par)] = dd
        for e, y in adj[x]:
            np_ = par ^ (1 if int(g.obs_mask[e]) >> bit & 1 else 0)
            nd = dd + int(g.w[e])
            if y < 0:
                if nd < bd.get((e, np_), 1 << 62):
                    bd[(e, np_)] = nd
            elif (y, np_) not in dist:
                heapq.heappush(h, (nd, y, np_))
    return dist, bd


def _definition_constrained(g, defects, bit=0):
    """(W0, W1) from the definition of the two constrained minima, without the
    chain rewrite: an edge set with odd degree exactly at the events splits
    into paths between events, paths from events to boundary vertices, paths
    between two boundary vertices and cycles.  Cycles carry no observable
    here (it sits on boundary edges only) and only add weight; two
    boundary-to-boundary paths of odd parity cancel.  So each minimum is the
    best pairing of the events (with each other or with the boundary) under
    parity-tracked shortest distances, with or without one boundary-to-boundary
    path of odd observable parity."""
    INF = 1 << 62
    m = len(defects)
    pair = [[[INF, INF] for _ in range(m)] for _ in range(m)]
    to_bd = [[INF, INF] for _ in range(m)]
    for i, s in enumerate(defects):
        dist, bd = _parity_search(g, bit, [(int(s), 0, 0)])
        for j, t in enumerate(defects):
            for par in (0, 1):
                pair[i][j][par] = dist.get((int(t), par), INF)
        for (e, par), dd in bd.items():
            to_bd[i][par] = min(to_bd[i][par], dd)
    # the cheapest boundary-to-boundary path of odd parity (two different boundary edges)
    bb = INF
    bedges = [e for e in range(g.num_edges) if int(g.v[e]) < 0]
    for e1 in bedges:
        p1 = int(g.obs_mask[e1]) >> bit & 1
        _, bd = _parity_search(g, bit, [(int(g.u[e1]), p1, int(g.w[e1]))])
        for (e2, par), dd in bd.items():
            if e2 != e1 and par == 1:
                bb = min(bb, dd)
    from functools import lru_cache

    @lru_cache(maxsize=None)
    def best(rest, par):
        if not rest:
            return 0 if par == 0 else INF
        i, others = rest[0], rest[1:]
        out = INF
        for q in (0, 1):
            if to_bd[i][q] < INF:
                out = min(out, to_bd[i][q] + best(others, par ^ q))
            for j in others:
                if pair[i][j][q] < INF:
                    out = min(out, pair[i][j][q] + best(tuple(x for x in others if x != j), par ^ q))
        return out

    res = []
    for target in (0, 1):
        v = min(best(tuple(range(m)), target),
                bb + best(tuple(range(m)), target ^ 1) if bb < INF else INF)
        res.append(None if v >= INF else v)
    return tuple(res)


@pytest.mark.parametrize("d,rounds,p", [(3, 3, 0.05), (5, 2, 0.03), (5, 5, 0.02)])
def test_complementary_equals_definition_without_the_rewrite(d, rounds, p):
    """Both constrained minima on rotated codes of 39 to 185 edges equal the
    parity-tracked pairing definition (no chain rewrite)."""
    g = synth.rotated_phenom_graph(d, p, rounds=rounds)
    assert g.num_edges > 16
    co = oracle.Complementary(g, 0, 0x5EED)
    s = synth.sample(g, 60, seed=31 + d)
    n = 0
    for i in range(60):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if len(dd) > 9:
            continue
        n += 1
        assert co.weights(dd) == _definition_constrained(g, dd.tolist()), (i, dd.tolist())
    assert n >= 30
