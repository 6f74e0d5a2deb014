"""Host checks of the synthetic detector graphs (no GPU)."""
import numpy as np

import synth


def test_circuit_x_graph_structure():
    """The circuit-level X-fault graph: degree within the decoder's 16, only
    positive weights, edges join the same or adjacent layers, it contains
    every phenomenological edge (a data fault before the round's first CNOT
    and a measurement error give exactly those), and faults between CNOTs
    add edges across layers (the diagonal mechanisms)."""
    d, p = 5, 0.001
    g = synth.rotated_circuit_x_graph(d, p)
    ph = synth.rotated_phenom_graph(d, p)
    nz = (d * d - 1) // 2
    deg = np.bincount(np.concatenate([g.u, g.v[g.v >= 0]]), minlength=g.num_detectors)
    assert deg.max() <= 16 and (g.w > 0).all()
    lu = g.u // nz
    inner = g.v >= 0
    lv = np.where(inner, g.v // nz, lu)
    assert (np.abs(lu - lv) <= 1).all()
    have = set(zip(g.u.tolist(), g.v.tolist()))
    for a, b in zip(ph.u.tolist(), ph.v.tolist()):
        assert (a, b) in have or (b, a) in have
    diag = [(a, b) for a, b in zip(g.u.tolist(), g.v.tolist()) if b >= 0 and a // nz != b // nz and a % nz != b % nz]
    assert len(diag) > 0
    assert len(set(g.w.tolist())) > 1


def test_circuit_x_graph_single_fault_counts():
    """Every mechanism merges the faults that flip the same detectors, so its
    probability is between p and 8p: the most an edge collects is a boundary
    edge of a plaquette with two one-plaquette data qubits, 4 fault slots
    each (m merged faults give (1 - (1 - 2p)^m) / 2 <= m p)."""
    p = 0.002
    g = synth.rotated_circuit_x_graph(7, p, rounds=4)
    assert (g.p >= p * (1 - 1e-9)).all() and (g.p <= 8 * p).all()
    assert g.p.max() > 7 * p


# ---- circuit-level X-memory graphs (both noise models of Methods, "Numerical evaluation")

from collections import deque

import pytest

from synth import circuit_level as cl


def _logical_distance(g):
    """Fewest edges in a boundary-to-boundary path with odd observable (BFS over (node, parity))."""
    B = g.num_detectors
    adj = [[] for _ in range(B + 1)]
    for a, b, o in zip(g.u.tolist(), g.v.tolist(), g.obs_mask.tolist()):
        b = B if b < 0 else b
        adj[a].append((b, o))
        adj[b].append((a, o))
    dist = {(B, 0): 0}
    todo = deque([(B, 0)])
    while todo:
        x, par = todo.popleft()
        for y, o in adj[x]:
            s = (y, par ^ o)
            if s not in dist:
                dist[s] = dist[(x, par)] + 1
                todo.append(s)
    return dist.get((B, 1))


def _x_face_incidence(d):
    """Data qubit (r, c) -> X faces holding it, from the face list alone."""
    inc = {}
    for i, (r, c) in enumerate(cl.x_faces(d)):
        for rr in (r, r + 1):
            for cc in (c, c + 1):
                if 0 <= rr < d and 0 <= cc < d:
                    inc.setdefault((rr, cc), []).append(i)
    return inc


@pytest.mark.parametrize("model", cl.NOISE_MODELS)
@pytest.mark.parametrize("d", [3, 5, 7, 9])
def test_circuit_graph_standard_schedule(model, d):
    """With the standard CNOT orders every detector is deterministic, every
    single fault is graphlike after CSS projection, detectors have degree at
    most 12 (the bound for circuit-level graphs), and the fewest faults that
    flip the logical observable undetected is d: the hook faults run across
    the logical operator, so the circuit keeps the code distance."""
    g = synth.rotated_circuit_graph(d, 0.001, model)
    nx = (d * d - 1) // 2
    assert g.num_detectors == nx * (d + 1)
    assert g.n_split == 0 and g.n_parallel == 0
    deg = np.bincount(np.concatenate([g.u, g.v[g.v >= 0]]), minlength=g.num_detectors)
    assert deg.max() == (12 if d >= 5 else 8) and (g.w > 0).all()
    assert _logical_distance(g) == d


@pytest.mark.parametrize("d", [5, 7])
def test_circuit_graph_hook_orientation_matters(d):
    """Exchanging the two plaquette types' CNOT orders turns the hook faults
    along the logical operator: the circuit distance falls to (d+1)/2."""
    g = synth.rotated_circuit_graph(d, 0.001, cnot_orders=(cl._ORDER_Z, cl._ORDER_X), parallel="keep_likelier")
    assert _logical_distance(g) == (d + 1) // 2


def test_circuit_graph_rejects_bad_schedules():
    """An order whose X and Z measurements do not commute leaves a detector
    that is not deterministic; an order that uses a qubit twice in a layer is
    not a circuit."""
    with pytest.raises(RuntimeError, match="deterministic"):
        synth.rotated_circuit_graph(5, 0.001, cnot_orders=(("NW", "NE", "SW", "SE"), ("SE", "NE", "SW", "NW")))
    with pytest.raises(ValueError, match="twice"):
        synth.rotated_circuit_graph(5, 0.001, cnot_orders=(("NW", "NE", "SW", "SE"), ("NW", "NE", "SE", "SW")))


def _merged(m, p):
    return (1.0 - (1.0 - 2.0 * p) ** m) / 2.0


@pytest.mark.parametrize("d,R", [(3, 3), (5, 4)])
def test_circuit_graph_measurement_flips_only(d, R):
    """Only measurement flips: an X-ancilla flip in round t is the timelike
    edge between layers t and t+1 of its face (Z-ancilla flips are invisible),
    and a flipped final data measurement is an edge in the last layer between
    the X faces holding that qubit, flipping the observable on column 0."""
    p = 0.003
    zero = {"prep": 0.0, "gate1": 0.0, "idle": 0.0, "cnot": 0.0}
    g = synth.rotated_circuit_graph(d, p, rounds=R, spec=dict(zero, meas=p))
    nx = (d * d - 1) // 2
    want = {}
    for t in range(1, R + 1):
        for i in range(nx):
            want[((t - 1) * nx + i, t * nx + i, 0)] = want.get(((t - 1) * nx + i, t * nx + i, 0), 0) + 1
    for (r, c), fs in _x_face_incidence(d).items():
        dets = sorted(R * nx + i for i in fs)
        key = (dets[0], dets[1] if len(dets) == 2 else -1, 1 if c == 0 else 0)
        want[key] = want.get(key, 0) + 1
    got = {(int(a), int(b), int(o)): q for a, b, o, q in zip(g.u, g.v, g.obs_mask, g.p)}
    assert set(got) == set(want)
    for k, m in want.items():
        assert got[k] == pytest.approx(_merged(m, p))


@pytest.mark.parametrize("d,R", [(3, 2), (5, 3)])
def test_circuit_graph_preparation_flips_only(d, R):
    """Only preparation flips: an X after an X ancilla's reset is turned into
    a measurement flip by the two Hadamards (timelike edge, as above), an X
    after a Z ancilla's reset is invisible, and a Z after a data qubit's X
    reset is an edge in layer 1 between the X faces holding it."""
    p = 0.002
    zero = {"meas": 0.0, "gate1": 0.0, "idle": 0.0, "cnot": 0.0}
    g = synth.rotated_circuit_graph(d, p, rounds=R, spec=dict(zero, prep=p))
    nx = (d * d - 1) // 2
    want = {}
    for t in range(1, R + 1):
        for i in range(nx):
            want[((t - 1) * nx + i, t * nx + i, 0)] = 1
    for (r, c), fs in _x_face_incidence(d).items():
        dets = sorted(fs)
        key = (dets[0], dets[1] if len(dets) == 2 else -1, 1 if c == 0 else 0)
        want[key] = want.get(key, 0) + 1
    got = {(int(a), int(b), int(o)): q for a, b, o, q in zip(g.u, g.v, g.obs_mask, g.p)}
    assert set(got) == set(want)
    for k, m in want.items():
        assert got[k] == pytest.approx(_merged(m, p))


def test_circuit_graph_merged_probabilities_bounded():
    """Each edge merges independent faults of probability at most p/3 (or p
    for preparation and measurement), so 0 < q < 1/2 and q never exceeds the
    sum of the model's per-location probabilities that can reach it."""
    p = 0.001
    for model in cl.NOISE_MODELS:
        g = synth.rotated_circuit_graph(7, p, model, rounds=5)
        assert (g.p > 0).all() and (g.p < 0.5).all()
        assert g.p.max() < 30 * p


def test_decompose_into_graphlike_parts():
    """The hyperedge split: parts are known graphlike faults whose
    observables XOR to the fault's own; None when no such split exists."""
    known = {(1, 2): (0,), (3, 4): (1,), (3,): (0,), (4,): (0,), (1, 3): (0,), (2, 4): (0, 1)}
    assert cl._decompose((1, 2, 3, 4), 1, known) == [((1, 2), 0), ((3, 4), 1)]
    assert cl._decompose((1, 2, 3, 4), 0, known) == [((1, 2), 0), ((3,), 0), ((4,), 0)]
    assert cl._decompose((1, 2, 5), 0, known) is None
    assert cl._decompose((2, 3, 4), 1, {(2,): (1,), (3, 4): (0,)}) == [((2,), 1), ((3, 4), 0)]


@pytest.mark.parametrize("model", cl.NOISE_MODELS)
@pytest.mark.parametrize("d,R", [(3, 4), (5, 5), (7, 3)])
def test_circuit_graph_windowed_scan_equals_full_scan(model, d, R):
    """Scanning only the detector layers near the current round gives the
    same graph as scanning every detector row (a detector's back-propagated
    frame lives in its own two rounds)."""
    a = synth.rotated_circuit_graph(d, 0.002, model, rounds=R)
    b = synth.rotated_circuit_graph(d, 0.002, model, rounds=R, windowed=False)
    for k in ("u", "v", "w", "obs_mask", "p"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
