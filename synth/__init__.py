"""Seeded synthetic inputs: rotated surface-code detector graphs and sampled shots.

This module is an input generator shared by the oracle and the GPU path.  It
builds the detector graph of the decoding task (Results, "Decoding task": one
vertex per detector, an edge per error that flips two detectors, and a fresh
boundary vertex with an edge per error that flips one detector) for the
rotated surface code under phenomenological noise, and it samples independent
edge flips.  It holds none of the decoding method's arithmetic.

Graph convention (d odd, d rounds, d+1 detector layers):
  * data qubits (r, c), 0 <= r, c < d;
  * Z-plaquettes are the interior faces (r', c'), 0 <= r', c' <= d-2 with
    r'+c' even, plus weight-2 faces on columns c' = -1 and c' = d-1 with
    r'+c' even; this gives (d^2-1)/2 detectors per layer;
  * an X flip of qubit (r, c) before measurement round t (t = 1..d) is a
    spatial edge in layer t between the faces containing that qubit; the 2d
    qubits of rows 0 and d-1 lie in a single face and give boundary edges;
  * a flipped measurement in round t (t = 1..d) is a timelike edge between
    layers t and t+1; layer d+1 comes from the noiseless final readout;
  * the observable (logical-Z crossing parity) is bit 0 of the mask of every
    row-0 boundary edge.
Edge order: spatial edges by (layer, r, c), then timelike edges by (t, face).
Boundary endpoints are written as -1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_sampler.so")


@dataclass
class DetectorGraph:
    """A detector graph with integer edge weights (host arrays)."""
    num_detectors: int
    u: np.ndarray          # int32 [E]
    v: np.ndarray          # int32 [E], -1 = own boundary vertex
    w: np.ndarray          # int32 [E], > 0
    obs_mask: np.ndarray   # uint64 [E]
    p: np.ndarray          # float64 [E], flip probability used by the sampler
    num_observables: int = 1
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.u.shape[0])

    @property
    def nbytes(self) -> int:
        return (self.num_detectors + 7) // 8


def weight_from_p(p: float) -> int:
    """Integer weight round(256 * ln((1-p)/p)), rounding half away from zero."""
    x = 256.0 * math.log((1.0 - p) / p)
    return int(math.floor(x + 0.5))


def z_faces(d: int):
    """Z-plaquettes of the distance-d rotated code, sorted by (r', c')."""
    faces = []
    for r in range(d - 1):
        for c in range(-1, d):
            if (r + c) % 2 != 0:
                continue
            if 0 <= c <= d - 2:
                q = [(r, c), (r + 1, c), (r, c + 1), (r + 1, c + 1)]
            elif c == -1:
                q = [(r, 0), (r + 1, 0)]
            else:  # c == d - 1
                q = [(r, d - 1), (r + 1, d - 1)]
            faces.append(((r, c), q))
    return faces


def rotated_phenom_graph(d: int, p: float, q: float | None = None,
                         w_spatial: int | None = None, w_time: int | None = None,
                         rounds: int | None = None) -> DetectorGraph:
    """Phenomenological rotated-code detector graph over `rounds` rounds (default d; rounds+1 layers of
    (d*d-1)/2 detectors, layer t holding detectors (t-1)*nz .. t*nz-1)."""
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    q = p if q is None else q
    ws = weight_from_p(p) if w_spatial is None else int(w_spatial)
    wt = weight_from_p(q) if w_time is None else int(w_time)
    faces = z_faces(d)
    nz = len(faces)
    assert nz == (d * d - 1) // 2
    qubit_faces: dict = {}
    for fi, (_, qs) in enumerate(faces):
        for qq in qs:
            qubit_faces.setdefault(qq, []).append(fi)
    R = d if rounds is None else int(rounds)
    if R < 1:
        raise ValueError("rounds must be >= 1")
    u, v, w, obs, pp = [], [], [], [], []
    for layer in range(1, R + 1):
        base = (layer - 1) * nz
        for r in range(d):
            for c in range(d):
                fs = qubit_faces[(r, c)]
                if len(fs) == 2:
                    u.append(base + fs[0]); v.append(base + fs[1])
                else:
                    assert len(fs) == 1 and r in (0, d - 1)
                    u.append(base + fs[0]); v.append(-1)
                w.append(ws); pp.append(p)
                obs.append(1 if (r == 0) else 0)
    for t in range(1, R + 1):
        for fi in range(nz):
            u.append((t - 1) * nz + fi); v.append(t * nz + fi)
            w.append(wt); pp.append(q); obs.append(0)
    return DetectorGraph(
        num_detectors=nz * (R + 1),
        u=np.asarray(u, np.int32), v=np.asarray(v, np.int32), w=np.asarray(w, np.int32),
        obs_mask=np.asarray(obs, np.uint64), p=np.asarray(pp, np.float64),
        name=f"rotated_phenom_d{d}_p{p}_q{q}")


def rotated_circuit_x_graph(d: int, p: float, rounds: int | None = None) -> DetectorGraph:
    """Detector graph of Z-basis memory on the rotated code from X faults in the syndrome-extraction circuit.

    Each round measures every Z plaquette with four CNOTs, data qubit as control and ancilla as target, in the
    order of the plaquette's qubit list (top-left, bottom-left, top-right, bottom-right; steps 1-4; the two
    weight-2 boundary plaquettes use steps 3-4 on the left edge and 1-2 on the right).  Fault mechanisms,
    each of probability p:
      * an X on a data qubit before CNOT step k+1 of round t (k = 0..3): plaquettes whose step for that
        qubit is later than k see it in round t (detector (t, P)), the others first in round t+1;
      * an X on a plaquette's ancilla before its measurement (a measurement error): detectors (t, P) and
        (t+1, P).
    Round 1 compares with the deterministic initial state and the final layer (rounds+1) with the
    transversal data measurement.  Mechanisms with the same detector pair merge (XOR of independent events:
    q = q1 + q2 - 2 q1 q2); weights are round(256 ln((1-q)/q)).  An X on a row-0 data qubit flips the
    logical observable."""
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    R = d if rounds is None else int(rounds)
    faces = z_faces(d)
    nz = len(faces)
    step = {}                                  # (qubit, face index) -> CNOT step 1..4
    for fi, ((r, c), qs) in enumerate(faces):
        steps = (1, 2, 3, 4) if len(qs) == 4 else ((3, 4) if c == -1 else (1, 2))
        for qq, st in zip(qs, steps):
            step[(qq, fi)] = st
    qubit_faces: dict = {}
    for (qq, fi) in step:
        qubit_faces.setdefault(qq, []).append(fi)
    mech: dict = {}                            # (u, v, obs) -> probability; v = -1 boundary

    def add(dets, obs):
        dets = sorted(set(dets))
        if not dets:
            return
        if len(dets) == 1:
            key = (dets[0], -1, obs)
        else:
            assert len(dets) == 2
            key = (dets[0], dets[1], obs)
        q0 = mech.get(key, 0.0)
        mech[key] = q0 + p - 2 * q0 * p

    for t in range(1, R + 1):
        for r in range(d):
            for c in range(d):
                fs = qubit_faces[(r, c)]
                for k in range(4):
                    dets = []
                    for fi in fs:
                        layer = t if step[((r, c), fi)] > k else t + 1
                        dets.append((layer - 1) * nz + fi)
                    add(dets, 1 if r == 0 else 0)
        for fi in range(nz):
            add([(t - 1) * nz + fi, t * nz + fi], 0)
    keys = sorted(mech)
    u = np.asarray([k[0] for k in keys], np.int32)
    v = np.asarray([k[1] for k in keys], np.int32)
    obs = np.asarray([k[2] for k in keys], np.uint64)
    pp = np.asarray([mech[k] for k in keys], np.float64)
    w = np.asarray([weight_from_p(float(q)) for q in pp], np.int32)
    return DetectorGraph(num_detectors=nz * (R + 1), u=u, v=v, w=w, obs_mask=obs, p=pp,
                         name=f"rotated_circuit_x_d{d}_p{p}_r{R}")


def repetition_graph(n_det: int, w, p: float = 0.01) -> DetectorGraph:
    """Path graph: boundary - 0 - 1 - ... - (n_det-1) - boundary (n_det+1 edges).

    Edge i joins detector i-1 and i (boundary for i = 0 and i = n_det).  The
    observable is carried by the left boundary edge.  Weights may be a scalar
    or a sequence of n_det+1 positive integers.
    """
    ne = n_det + 1
    ww = np.full(ne, int(w), np.int32) if np.isscalar(w) else np.asarray(w, np.int32)
    u = np.empty(ne, np.int32); v = np.empty(ne, np.int32)
    u[0], v[0] = 0, -1
    for i in range(1, n_det):
        u[i], v[i] = i - 1, i
    u[n_det], v[n_det] = n_det - 1, -1
    obs = np.zeros(ne, np.uint64); obs[0] = 1
    return DetectorGraph(n_det, u, v, ww, obs, np.full(ne, p), name=f"repetition_{n_det}")


def random_graph(n_det: int, n_edges: int, n_boundary: int, wmin: int, wmax: int, seed: int,
                 p: float = 0.05) -> DetectorGraph:
    """Random connected graph with boundary edges (a spanning path keeps it connected)."""
    rng = np.random.default_rng(seed)
    pairs = set()
    perm = rng.permutation(n_det)
    for i in range(n_det - 1):
        a, b = int(perm[i]), int(perm[i + 1])
        pairs.add((min(a, b), max(a, b)))
    while len(pairs) < n_edges - n_boundary:
        a, b = rng.integers(0, n_det, 2)
        if a != b:
            pairs.add((int(min(a, b)), int(max(a, b))))
    u = [a for a, _ in sorted(pairs)]
    v = [b for _, b in sorted(pairs)]
    for _ in range(n_boundary):
        u.append(int(rng.integers(0, n_det))); v.append(-1)
    ne = len(u)
    w = rng.integers(wmin, wmax + 1, ne).astype(np.int32)
    obs = rng.integers(0, 4, ne).astype(np.uint64)
    return DetectorGraph(n_det, np.asarray(u, np.int32), np.asarray(v, np.int32), w, obs,
                         np.full(ne, p), num_observables=2, name=f"random_{n_det}_{seed}")


def _lib():
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, "sampler.c")):
        build()
    lib = ctypes.CDLL(_SO)
    lib.synth_sample.restype = ctypes.c_int
    return lib


def build() -> None:
    """Compile the sampler (plain C, host only)."""
    src = os.path.join(_HERE, "sampler.c")
    tmp = _SO + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, _SO)


@dataclass
class Shots:
    syndromes: np.ndarray   # uint8 [n, nbytes]
    obs: np.ndarray         # uint64 [n], observable flips of the hidden error
    weight: np.ndarray      # int64 [n], weight of the hidden error
    seed: int
    shot0: int


def sample(g: DetectorGraph, n: int, seed: int, shot0: int = 0) -> Shots:
    """Sample n shots (global shot indices shot0 .. shot0+n-1) from the seeded stream."""
    thr = np.floor(g.p * 4294967296.0).astype(np.uint64)
    thr = np.minimum(thr, 4294967295).astype(np.uint32)
    synd = np.zeros((n, g.nbytes), np.uint8)
    obs = np.zeros(n, np.uint64)
    wt = np.zeros(n, np.int64)
    P = ctypes.c_void_p
    rc = _lib().synth_sample(
        ctypes.c_int64(g.num_edges), P(g.u.ctypes.data), P(g.v.ctypes.data), P(thr.ctypes.data),
        P(g.obs_mask.ctypes.data), P(g.w.ctypes.data), ctypes.c_int32(g.num_detectors),
        ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ctypes.c_int64(shot0), ctypes.c_int64(n),
        P(synd.ctypes.data), P(obs.ctypes.data), P(wt.ctypes.data))
    if rc != 0:
        raise RuntimeError("synth_sample failed")
    return Shots(synd, obs, wt, seed, shot0)


def syndrome_from_edges(g: DetectorGraph, edges) -> np.ndarray:
    """Packed syndrome row of an explicit edge set (for hand-built cases)."""
    row = np.zeros(g.nbytes, np.uint8)
    for e in edges:
        for x in (int(g.u[e]), int(g.v[e])):
            if x >= 0:
                row[x >> 3] ^= np.uint8(1 << (x & 7))
    return row


def defects_of(row: np.ndarray, num_detectors: int) -> np.ndarray:
    """Sorted detector ids whose bit is set in a packed syndrome row."""
    bits = np.unpackbits(row, bitorder="little")[:num_detectors]
    return np.nonzero(bits)[0].astype(np.int32)


def rotated_circuit_graph(d: int, p: float, model: str = "uniform", rounds: int | None = None, **kw) -> DetectorGraph:
    """Circuit-level detector graph of X-basis memory on the rotated code (uniform or physical noise
    model); defined in synth.circuit_level."""
    from .circuit_level import rotated_circuit_graph as _build
    return _build(d, p, model, rounds, **kw)
