"""Pins for the serial sparse-blossom oracle (``oracle.SparseBlossom``):
global sparse blossom and partition-and-fuse must return the MWEM of the
Dijkstra + Edmonds oracle on every shot (Theorem 1: the same result as global
sparse blossom, which computes an MWEM), the event counts and E_ideal of small
hand-worked cases follow from the dynamics by hand, and the C clustering equals
the plain definition in ``oracle.cluster_levels``."""
import multiprocessing as mp

import numpy as np
import pytest

import oracle
import synth

SEED = 0x5EED


def _schedule(og, levels=8):
    d, b, _ = oracle.schedule(max(og.tiebroken_weights()), levels=levels)
    return d, b


def _check_shots(g, syndromes, idx, reading="strict"):
    """Shots (from idx) where global or partition-and-fuse sparse blossom
    differs from the MWEM, or raises a flag, or where the two disagree on the
    event counts."""
    og = oracle.Graph(g, SEED)
    sb = oracle.SparseBlossom(g, SEED)
    d, b = _schedule(og)
    bad = []
    for i in idx:
        dd = synth.defects_of(syndromes[i], g.num_detectors)
        r = og.mwem(dd)
        pf = sb.decode(dd, d, b, reading=reading)
        gl = sb.decode(dd, global_mode=True)
        if r.flags & oracle.OF_INFEASIBLE:
            if not (pf.flags & oracle.SBF_INFEASIBLE) or not (gl.flags & oracle.SBF_INFEASIBLE):
                bad.append((i, "infeasible expected", pf.flags, gl.flags))
            continue
        for name, s in (("pf", pf), ("global", gl)):
            if s.flags or s.edges.tolist() != r.edges.tolist() or s.weight != r.weight or s.obs != r.obs:
                bad.append((i, name, len(dd), s.flags, s.weight, r.weight))
        # the partitioned run replays the global dynamics cluster by cluster (Theorem 1's proof):
        # the same events happen, and in global mode everything is one cluster
        if (pf.events, pf.arrivals) != (gl.events, gl.arrivals) or gl.e_ideal != gl.events or pf.e_ideal > pf.events:
            bad.append((i, "counts", pf.events, gl.events, pf.arrivals, gl.arrivals, pf.e_ideal, gl.e_ideal))
    return bad


_POOL_ARGS = None


def _pool_init(g, syndromes):
    global _POOL_ARGS
    _POOL_ARGS = (g, syndromes)


def _pool_chunk(idx):
    g, syndromes = _POOL_ARGS
    return _check_shots(g, syndromes, idx)


def _check_parallel(g, syndromes, chunk=2000, workers=8):
    n = syndromes.shape[0]
    parts = [list(range(s, min(n, s + chunk))) for s in range(0, n, chunk)]
    with mp.get_context("fork").Pool(workers, initializer=_pool_init, initargs=(g, syndromes)) as pool:
        bad = []
        for b in pool.imap(_pool_chunk, parts):
            bad.extend(b)
    return bad


# ---------------------------------------------------------------- every shot of the two small configurations
def test_config1_every_shot_equals_mwem():
    """d=5, 5 rounds, p=q=0.005: all 10,000 shots."""
    g = synth.rotated_phenom_graph(5, 0.005)
    s = synth.sample(g, 10000, seed=1)
    assert _check_shots(g, s.syndromes, range(10000)) == []


def test_config2_every_shot_equals_mwem():
    """d=11, 11 rounds, p=q=0.003: all 100,000 shots (spread over host processes)."""
    g = synth.rotated_phenom_graph(11, 0.003)
    s = synth.sample(g, 100000, seed=2)
    assert _check_parallel(g, s.syndromes) == []


@pytest.mark.parametrize("p,seed,n", [(0.005, 3, 24), (0.001, 4, 120)])
def test_d21_sample_equals_mwem(p, seed, n):
    g = synth.rotated_phenom_graph(21, p)
    s = synth.sample(g, n, seed=seed)
    assert _check_shots(g, s.syndromes, range(n)) == []


@pytest.mark.parametrize("d,p,n,seed", [(9, 0.03, 200, 7), (7, 0.06, 200, 8), (5, 0.12, 300, 9)])
def test_high_error_rates_blossoms(d, p, n, seed):
    """Dense syndromes: blossoms form, shatter and implode often."""
    g = synth.rotated_phenom_graph(d, p)
    s = synth.sample(g, n, seed=seed)
    assert _check_shots(g, s.syndromes, range(n)) == []
    assert _check_shots(g, s.syndromes, range(0, n, 3), reading="loose") == []


@pytest.mark.parametrize("model,d,p,n", [("uniform", 5, 0.004, 300), ("physical", 5, 0.006, 300)])
def test_circuit_level_graphs(model, d, p, n):
    """Non-uniform weights, degree up to 12, diagonal spacetime edges."""
    g = synth.rotated_circuit_graph(d, p, model)
    s = synth.sample(g, n, seed=11)
    assert _check_shots(g, s.syndromes, range(n)) == []


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_with_random_syndromes(seed):
    """Random connected graphs with mixed weights and random defect sets."""
    g = synth.random_graph(40, 90, 6, 1, 9, seed=seed)
    rng = np.random.default_rng(100 + seed)
    rows = []
    for _ in range(60):
        k = int(rng.integers(0, 14))
        row = np.zeros(g.nbytes, np.uint8)
        for x in rng.choice(g.num_detectors, k, replace=False):
            row[x >> 3] |= np.uint8(1 << (x & 7))
        rows.append(row)
    assert _check_shots(g, np.stack(rows), range(60)) == []


# ---------------------------------------------------------------- hand-worked dynamics
def _path(ws, defects, **kw):
    g = synth.repetition_graph(len(ws) - 1, ws)
    og = oracle.Graph(g, SEED)
    d, b = _schedule(og, 6)
    return oracle.SparseBlossom(g, SEED).decode(np.asarray(defects, np.int32), d, b, **kw)


def test_event_counts_and_e_ideal_worked_example_overlap():
    """Path boundary-0-1-...-19-boundary; boundary edges weight 10, inner edges
    weight 9 (doubled: 20 and 18).  Events at detectors 0, 8, 11.

    Level 1: {0} (its boundary vertex is within d_1 = w_max + 1; 8 is more than
    b_1 away).  {8, 11} are three edges apart (54 > b_1 = 2 d_1 + 1), so they
    are level 2 (diameter 54 <= d_2, even).
    Level 1 run: region 0 enters detector 1 at t=18 (ARRIVE), meets the
    boundary at t=20 (COLLIDE): 2 events, s(C1)=20, so t_<2 = 20, E_<2 = 2.
    Level 2 run: regions 8 and 11 enter 7, 9, 10, 12 at t=18 (4 ARRIVE), and
    meet across edge (9, 10) at t = 18 + 18/2 = 27 (COLLIDE): 5 events, 4 of
    them at t <= t_<2.  E(C2) = max(2, 4) + 5 - 4 = 5.  Total 7 events, of
    which 5 ARRIVE."""
    ws = [10] + [9] * 19 + [10]
    pf = _path(ws, [0, 8, 11])
    assert pf.flags == 0
    assert pf.levels.tolist() == [1, 2, 2]
    assert (pf.events, pf.arrivals, pf.e_ideal, pf.clusters, pf.max_level) == (7, 5, 5, 2, 2)
    assert pf.edges.tolist() == [0, 9, 10, 11]           # boundary edge of 0, path 8-9-10-11
    gl = _path(ws, [0, 8, 11], global_mode=True)
    assert (gl.events, gl.arrivals, gl.e_ideal, gl.clusters) == (7, 5, 7, 1)
    # level-1 exploring regions (radius b_1/2, just above one edge): {0, 1}, {7, 8, 9}, {10, 11, 12}
    assert pf.level1_search == 8


def test_event_counts_and_e_ideal_worked_example_no_overlap():
    """The same events with inner edges of weight 11 (doubled 22): region 0
    meets the boundary at t=20 before it could enter detector 1 (t=22), so
    C1 has 1 event and t_<2 = 20.  {8, 11} (66 > b_1 = 47 apart) enter
    7, 9, 10, 12 at t=22 and collide at t=33: 5 events, none by t=20, so
    E(C2) = max(1, 0) + 5 - 0 = 6 = all events."""
    ws = [10] + [11] * 19 + [10]
    pf = _path(ws, [0, 8, 11])
    assert pf.levels.tolist() == [1, 2, 2]
    assert (pf.events, pf.arrivals, pf.e_ideal, pf.clusters, pf.max_level) == (6, 4, 6, 2, 2)


def test_single_event_far_from_the_boundary_strict_and_loose():
    """One event at detector 30 of a 60-detector path (weights 10): the region
    fills 29 detectors on the left and 29 on the right (58 ARRIVE) and meets
    the right boundary after 30 edges (COLLIDE): 59 events, all on the
    critical path.  The event is 30 edges (600) from its nearest boundary
    vertex: beyond d_2 = 3 d_1 + 4 b_1 + 2 w_max (about 13 edges), so the
    strict reading accepts it only at level 3; b_2/2 (hundreds of edges)
    reaches the boundary, so the loose reading accepts it at level 2."""
    ws = [10] * 61
    st = _path(ws, [30])
    lo = _path(ws, [30], reading="loose")
    assert st.levels.tolist() == [3] and lo.levels.tolist() == [2]
    for r in (st, lo):
        assert (r.events, r.arrivals, r.e_ideal, r.clusters) == (59, 58, 59, 1)
        assert r.edges.tolist() == list(range(31, 61))
    # the plain definition agrees
    g = synth.repetition_graph(60, ws)
    og = oracle.Graph(g, SEED)
    d, b = _schedule(og, 6)
    D, _ = og.defect_distances([30])
    BT = og.boundary_table([30])
    assert oracle.cluster_levels(D, BT, d, b, "strict") == [3]
    assert oracle.cluster_levels(D, BT, d, b, "loose") == [2]


def test_isolated_pair_and_boundary_singleton_single_events():
    """An adjacent pair collides once (t = 10); a singleton whose boundary edge
    (weight 9) is lighter than its inner edge (weight 10) meets the boundary
    (t = 18) before it could enter its neighbour (t = 20): each a level-1
    cluster of one event."""
    ws = [10] * 30 + [9]
    r = _path(ws, [5, 6, 29])
    assert r.levels.tolist() == [1, 1, 1]
    assert (r.events, r.arrivals, r.e_ideal, r.clusters, r.max_level) == (2, 0, 1, 2, 1)
    assert r.edges.tolist() == [6, 30]
    assert _path(ws, []).events == 0


# ---------------------------------------------------------------- clustering: C against the plain definition
@pytest.mark.parametrize("reading", ["strict", "loose"])
def test_c_clustering_equals_definition(reading):
    cases = []
    g = synth.rotated_phenom_graph(7, 0.02)
    s = synth.sample(g, 40, seed=21)
    cases += [(g, synth.defects_of(s.syndromes[i], g.num_detectors)) for i in range(40)]
    for seed in range(4):
        gr = synth.random_graph(30, 70, 5, 1, 9, seed=seed)
        rng = np.random.default_rng(seed)
        for _ in range(10):
            cases.append((gr, np.sort(rng.choice(30, int(rng.integers(1, 10)), replace=False)).astype(np.int32)))
    for g, dd in cases:
        if len(dd) == 0:
            continue
        og = oracle.Graph(g, SEED)
        d, b = _schedule(og, 6)
        D, _ = og.defect_distances(dd)
        BT = og.boundary_table(dd)
        lv, comps = oracle.cluster_levels(D, BT, d, b, reading, components=True)
        r = oracle.SparseBlossom(g, SEED).decode(dd, d, b, reading=reading)
        assert r.levels.tolist() == lv
        assert r.clusters == len(comps) and r.max_level == max(lv)
