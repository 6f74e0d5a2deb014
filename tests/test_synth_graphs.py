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
