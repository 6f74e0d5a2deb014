"""Circuit-level detector graphs of the rotated surface code (X-basis memory).

Input generator only: it derives the weighted detector graph that the decoder
is handed, and holds none of the decoding method's arithmetic.

Experiment (Methods, "Numerical evaluation"): the logical qubit is prepared in
|+>_L, measured by `rounds` rounds of syndrome extraction, then every data
qubit is measured in the X basis.  The decoding graph holds the X-type
detectors; Z components of faults flip them (the CSS projection of each
fault).  Two noise models, both parameterised by p:
  * "uniform": a prepared state flips with p; after every single-qubit gate,
    idling included, X, Y and Z each occur with p/3; after every CNOT each of
    the 15 non-identity two-qubit Paulis occurs with p/15; a measurement
    outcome flips with p;
  * "physical": as "uniform", but non-idle single-qubit gates get p/30 per
    Pauli and idling is noiseless.

Circuit, per round, eight moments (every qubit is acted on or idles in each):
  0  reset every ancilla in Z (in the first syndrome round the data are also
     reset in X in this moment)
  1  H on the X ancillas
  2-5  four CNOT layers: X ancilla -> data in the order NW, NE, SW, SE;
       data -> Z ancilla in the order NW, SW, NE, SE
  6  H on the X ancillas
  7  measure every ancilla in Z
then the data are measured in X.  A face (r, c) covers data (r, c) NW,
(r, c+1) NE, (r+1, c) SW, (r+1, c+1) SE, those inside the d x d grid.

Detectors (layer t = 1..rounds+1, nx = (d^2-1)/2 per layer, detector
(t-1)*nx + i for X face i): layer 1 is the first measurement of each X
ancilla, layer t in 2..rounds compares rounds t-1 and t, layer rounds+1
compares the last round with the product of that face's data X measurements.
The observable is the X measurement parity of data column 0 (the logical X).

Fault effects come from propagating every detector (and the observable)
backwards through the circuit as a Pauli frame: a fault flips a detector
exactly when it anticommutes with that detector's back-propagated Pauli at the
fault's location.  A reset absorbs the component it stabilises; any other
component left at a reset means the detector is not deterministic, which is
an error.  Faults with the same effect merge (XOR of independent events,
q = q1 + q2 - 2 q1 q2).  A fault flipping more than two detectors is split
into detector pairs and singletons that single faults also produce, their
observables summing to its own; its probability is merged into each part.
Parallel edges with different observables are an error (or, on request, keep the more probable one).
Weights are round(256 ln((1-q)/q)).  Edges are independent in the sampler,
so the correlations of split faults are not reproduced in sampled shots.
"""
from __future__ import annotations

import numpy as np

_ORDER_X = ("NW", "NE", "SW", "SE")
_ORDER_Z = ("NW", "SW", "NE", "SE")
_CORNER = {"NW": (0, 0), "NE": (0, 1), "SW": (1, 0), "SE": (1, 1)}

NOISE_MODELS = ("uniform", "physical")


def x_faces(d: int):
    """X-plaquettes of the distance-d rotated code, sorted by (r', c'): interior faces with r'+c' odd and
    weight-2 faces on rows -1 and d-1."""
    out = []
    for r in range(-1, d):
        for c in range(d - 1):
            if (r + c) % 2 == 1:
                out.append((r, c))
    return out


def _z_face_corners(d: int):
    out = []
    for r in range(d - 1):
        for c in range(-1, d):
            if (r + c) % 2 == 0:
                out.append((r, c))
    return out


def _face_steps(d: int, rc, order):
    """(step 1..4, data (r, c)) of one face, for the corners inside the grid."""
    r, c = rc
    out = []
    for k, name in enumerate(order):
        dr, dc = _CORNER[name]
        rr, cc = r + dr, c + dc
        if 0 <= rr < d and 0 <= cc < d:
            out.append((k + 1, (rr, cc)))
    return out


def noise_spec(model: str, p: float) -> dict:
    """Per-location probabilities of the two noise models (see module docstring)."""
    if model == "uniform":
        return {"prep": p, "meas": p, "gate1": p / 3, "idle": p / 3, "cnot": p / 15}
    if model == "physical":
        return {"prep": p, "meas": p, "gate1": p / 30, "idle": 0.0, "cnot": p / 15}
    raise ValueError(f"unknown noise model {model!r}")


class _Frames:
    """Back-propagated Pauli frames, one column per detector row (and the observable row last)."""

    def __init__(self, nq: int, nrows: int):
        self.x = np.zeros((nq, nrows), np.bool_)
        self.z = np.zeros((nq, nrows), np.bool_)
        self.obs_row = nrows - 1
        self.mech: dict = {}
        self.lo, self.hi = 0, nrows - 1   # detector rows that can be non-zero now (the observable row always)

    def _rows(self, col):
        r = (np.flatnonzero(col[self.lo:self.hi]) + self.lo).tolist()
        if col[self.obs_row]:
            r.append(self.obs_row)
        return frozenset(r)

    # effects of single-qubit Pauli components at the current time
    def _hits(self, q: int):
        return self._rows(self.z[q]), self._rows(self.x[q])   # rows an X on q flips, rows a Z on q flips

    def _add(self, rows: frozenset, prob: float):
        if not rows or prob <= 0.0:
            return
        obs = 1 if self.obs_row in rows else 0
        dets = tuple(sorted(r for r in rows if r != self.obs_row))
        key = (dets, obs)
        q0 = self.mech.get(key, 0.0)
        self.mech[key] = q0 + prob - 2.0 * q0 * prob

    def flip_x(self, q, prob):
        if prob > 0:
            self._add(self._hits(q)[0], prob)

    def flip_z(self, q, prob):
        if prob > 0:
            self._add(self._hits(q)[1], prob)

    def dep1(self, q, prob):
        if prob <= 0:
            return
        hx, hz = self._hits(q)
        self._add(hx, prob); self._add(hz, prob); self._add(hx ^ hz, prob)

    def dep2(self, a, b, prob):
        if prob <= 0:
            return
        ax, az = self._hits(a)
        bx, bz = self._hits(b)
        pa = (frozenset(), ax, ax ^ az, az)       # I, X, Y, Z on a
        pb = (frozenset(), bx, bx ^ bz, bz)
        for i in range(4):
            for j in range(4):
                if i or j:
                    self._add(pa[i] ^ pb[j], prob)

    # gates, applied backwards (each is its own inverse under conjugation)
    def cx(self, ctl, tgt):
        self.x[tgt] ^= self.x[ctl]
        self.z[ctl] ^= self.z[tgt]

    def h(self, qs):
        tmp = self.x[qs].copy()
        self.x[qs] = self.z[qs]
        self.z[qs] = tmp

    def reset_z(self, qs):
        if self.x[qs].any():
            raise RuntimeError("a detector is not deterministic (X component at a Z reset)")
        self.z[qs] = False

    def reset_x(self, qs):
        if self.z[qs].any():
            raise RuntimeError("a detector is not deterministic (Z component at an X reset)")
        self.x[qs] = False


def _decompose(dets, obs, graphlike):
    """Split a detector set into graphlike parts (pairs or singletons) that single faults produce, whose
    observables XOR to `obs`; None if there is no such split.  Deterministic: the lowest detector is covered
    first, pairs before singletons, partners in increasing order."""
    if not dets:
        return [] if obs == 0 else None
    a = dets[0]
    rest = dets[1:]
    options = []
    for b in rest:
        options.append(((a, b), tuple(x for x in rest if x != b)))
    options.append(((a,), rest))
    for part, remaining in options:
        for o in graphlike.get(part, ()):
            sub = _decompose(remaining, obs ^ o, graphlike)
            if sub is not None:
                return [(part, o)] + sub
    return None


def rotated_circuit_graph(d: int, p: float, model: str = "uniform", rounds: int | None = None,
                          spec: dict | None = None, cnot_orders=(_ORDER_X, _ORDER_Z), windowed: bool = True,
                          parallel: str = "raise"):
    """Detector graph of the X-basis memory experiment under a circuit-level noise model.

    `spec` overrides the per-location probabilities ({"prep", "meas", "gate1", "idle", "cnot"}, each the
    probability of one Pauli term), for special cases.  `cnot_orders` gives the corner order of the X and
    of the Z plaquettes' CNOTs (default: the schedule in the module docstring); an order that uses a qubit
    twice in one layer raises ValueError, one whose measurements do not commute raises RuntimeError.
    `windowed` scans, while round t is propagated, only the rows of detector layers t-1..t+2 (and the
    observable): a layer-L detector's frame lives in rounds L-1 and L only, since every reset of the round
    before absorbs it.  windowed=False scans every row (for checking that claim).
    Two faults with the same detectors but different observable flips would be parallel edges, which a
    detector graph cannot hold: `parallel="raise"` (default) raises ValueError for them, and
    `parallel="keep_likelier"` keeps the more probable one and counts the other.
    Returns a DetectorGraph (synth.DetectorGraph) with two more attributes: `n_split` (faults split into
    parts) and `n_parallel` (parallel edges dropped)."""
    from . import DetectorGraph, weight_from_p
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    R = d if rounds is None else int(rounds)
    if R < 1:
        raise ValueError("rounds must be >= 1")
    ns = noise_spec(model, p) if spec is None else dict(spec)
    xf = x_faces(d)
    zf = _z_face_corners(d)
    nx = len(xf)
    assert nx == (d * d - 1) // 2 and len(zf) == nx
    nd = d * d
    xa = [nd + i for i in range(nx)]
    za = [nd + nx + j for j in range(len(zf))]
    nq = nd + 2 * nx
    data = list(range(nd))

    def dq(rc):
        return rc[0] * d + rc[1]

    # CNOT layers: step -> list of (control, target)
    layers = {k: [] for k in (1, 2, 3, 4)}
    order_x, order_z = (tuple(o) for o in cnot_orders)
    for o in (order_x, order_z):
        if sorted(o) != sorted(_CORNER):
            raise ValueError("a CNOT order must list NW, NE, SW and SE once each")
    for i, rc in enumerate(xf):
        for k, dd in _face_steps(d, rc, order_x):
            layers[k].append((xa[i], dq(dd)))
    for j, rc in enumerate(zf):
        for k, dd in _face_steps(d, rc, order_z):
            layers[k].append((dq(dd), za[j]))
    for k in layers:
        used = [q for pair in layers[k] for q in pair]
        if len(used) != len(set(used)):
            raise ValueError("a qubit is used twice in one CNOT layer")
    x_faces_of = {q: [] for q in data}
    for i, rc in enumerate(xf):
        for _, dd in _face_steps(d, rc, order_x):
            x_faces_of[dq(dd)].append(i)

    nrows = nx * (R + 1) + 1
    F = _Frames(nq, nrows)
    allq = list(range(nq))

    def idle(busy):
        if ns["idle"] > 0:
            b = set(busy)
            for q in allq:
                if q not in b:
                    F.dep1(q, ns["idle"])

    # final X measurement of the data: include it, then the flip before it
    if windowed:
        F.lo = max(0, (R - 1) * nx)
    for q in data:
        rows = [R * nx + i for i in x_faces_of[q]]
        if q % d == 0:
            rows.append(F.obs_row)
        F.x[q, rows] ^= True
    for q in data:
        F.flip_z(q, ns["meas"])

    anc = xa + za
    for t in range(R, 0, -1):
        if windowed:
            F.lo, F.hi = max(0, (t - 2) * nx), min(nrows - 1, (t + 2) * nx)
        # moment 7: measure ancillas in Z (data idle)
        idle(anc)
        for i, a in enumerate(xa):
            rows = [(t - 1) * nx + i, t * nx + i]
            F.z[a, rows] ^= True
        for a in anc:
            F.flip_x(a, ns["meas"])
        # moment 6: H on X ancillas
        for a in xa:
            F.dep1(a, ns["gate1"])
        idle(xa)
        F.h(xa)
        # moments 5..2: CNOT layers 4..1
        for k in (4, 3, 2, 1):
            busy = []
            for (c_, t_) in layers[k]:
                F.dep2(c_, t_, ns["cnot"])
                busy += [c_, t_]
            idle(busy)
            for (c_, t_) in layers[k]:
                F.cx(c_, t_)
        # moment 1: H on X ancillas
        for a in xa:
            F.dep1(a, ns["gate1"])
        idle(xa)
        F.h(xa)
        # moment 0: reset ancillas (and, in the first syndrome round, the data in X)
        for a in anc:
            F.flip_x(a, ns["prep"])
        if t == 1:
            for q in data:
                F.flip_z(q, ns["prep"])
            F.reset_z(anc)
            F.reset_x(data)
        else:
            idle(anc)
            F.reset_z(anc)
    if F.x.any() or F.z.any():
        raise RuntimeError("a detector is not deterministic (frame left before the first reset)")

    # graphlike faults, then split the others
    graphlike: dict = {}
    for (dets, obs), q in F.mech.items():
        if dets and len(dets) <= 2:
            graphlike.setdefault(dets, set()).add(obs)
    graphlike = {k: tuple(sorted(v)) for k, v in graphlike.items()}
    edges: dict = {}

    def merge(key, q):
        q0 = edges.get(key, 0.0)
        edges[key] = q0 + q - 2.0 * q0 * q

    n_split = 0
    for (dets, obs), q in sorted(F.mech.items()):
        if not dets:
            if obs:
                raise RuntimeError("a single fault flips the observable undetected")
            continue
        if len(dets) <= 2:
            merge((dets, obs), q)
            continue
        parts = _decompose(dets, obs, graphlike)
        if parts is None:
            raise RuntimeError(f"fault with detectors {dets} has no graphlike split")
        n_split += 1
        for part, o in parts:
            merge((part, o), q)
    # parallel edges with different observables: keep the more probable
    best: dict = {}
    for (dets, obs), q in edges.items():
        cur = best.get(dets)
        if cur is None or q > cur[1] or (q == cur[1] and obs < cur[0]):
            best[dets] = (obs, q)
    n_parallel = len(edges) - len(best)
    if n_parallel and parallel != "keep_likelier":
        raise ValueError(f"{n_parallel} pairs of faults share their detectors but differ in the observable "
                         "(pass parallel='keep_likelier' to keep the more probable of each)")
    keys = sorted(best)
    u = np.asarray([k[0] for k in keys], np.int32)
    v = np.asarray([k[1] if len(k) == 2 else -1 for k in keys], np.int32)
    obs_a = np.asarray([best[k][0] for k in keys], np.uint64)
    pp = np.asarray([best[k][1] for k in keys], np.float64)
    w = np.asarray([weight_from_p(float(q)) for q in pp], np.int32)
    if (w <= 0).any():
        raise ValueError("an edge probability is >= 1/2")
    g = DetectorGraph(num_detectors=nx * (R + 1), u=u, v=v, w=w, obs_mask=obs_a, p=pp,
                      name=f"rotated_circuit_{model}_d{d}_r{R}_p{p}_split{n_split}_parallel{n_parallel}")
    g.n_split = n_split
    g.n_parallel = n_parallel
    return g
