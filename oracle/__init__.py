"""ORACLE -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It is a plain, slow CPU computation of
what the decoder computes, written from the paper, and shares no code with the
GPU path (``paper_2609_12262_amd``); the two meet only in the seeded input
generator ``synth``.

Contents:
  * ``mwem``            -- minimum-weight embedded matching of one shot
                           (Results, "Decoding task"): Dijkstra + Edmonds on the
                           defect graph with an LP certificate (Supplementary S1),
                           in ``mwem.c``.
  * ``SparseBlossom``   -- serial global sparse blossom (Supplementary S1) and
                           serial partition-and-fuse (Methods: Algorithm
                           "Clustering", the hierarchical execution rule,
                           Algorithm "Parallel sparse blossom") with the event
                           counts and the parallel event count E_ideal (Methods,
                           numerical evaluation), in ``sparse_blossom.c``.
  * ``schedule``        -- finite-size parameter schedule (Methods, Algorithm
                           "Parameter schedule"; Supplementary S11), exact rationals.
  * ``cluster_levels``  -- processing-cluster hierarchy (Methods, Algorithm
                           "Clustering"), from exact pairwise distances.
  * ``window_schedule``,
    ``window_decode``   -- sliding-window decoding of a layered graph
                           (Introduction: a stream of rounds decoded in
                           overlapping windows), each window by ``mwem``.
  * ``Complementary``   -- minimum weight under each value of one logical
                           observable and their gap (Introduction: the
                           complementary gap), each an MWEM of a rewritten graph.
  * ``brute_*``         -- brute-force pins for tiny inputs.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")

OF_TIE, OF_INFEASIBLE, OF_CERT_FAIL, OF_CAPACITY = 1, 2, 4, 8
INF_HI = np.iinfo(np.int64).max


_SRCS = ("mwem.c", "sparse_blossom.c")


def build() -> None:
    """Compile the C part of the oracle (gcc, host only)."""
    tmp = _SO + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, *[os.path.join(_HERE, f) for f in _SRCS]])
    os.replace(tmp, _SO)


_lib_cache = None


def _lib():
    global _lib_cache
    if _lib_cache is None:
        if not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, f))
                                          for f in _SRCS):
            build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_graph_create.restype = ctypes.c_void_p
        lib.oracle_graph_destroy.argtypes = [ctypes.c_void_p]
        for name in ("oracle_mwem", "oracle_dijkstra", "oracle_defect_distances",
                     "oracle_defect_boundary_table", "oracle_max_weight_matching", "oracle_sb_decode"):
            getattr(lib, name).restype = ctypes.c_int
        lib.oracle_sb_graph_create.restype = ctypes.c_void_p
        lib.oracle_sb_graph_destroy.argtypes = [ctypes.c_void_p]
        _lib_cache = lib
    return _lib_cache


def _p(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _join(hi: np.ndarray, lo: np.ndarray):
    """Exact Python ints from (hi, lo) halves; INF_HI -> None."""
    out = []
    for h, l in zip(hi.tolist(), lo.tolist()):
        out.append(None if h == INF_HI else (int(h) << 64) + int(l))
    return out


def splitmix_output(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 seeded with `seed` (Steele, Lea & Flood 2014)."""
    m = (1 << 64) - 1
    z = (seed + k * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def tiebroken_weight(w: int, seed: int, e: int) -> int:
    """wt(e) = 2 w(e) 2^64 + 2 h(e), h(e) = output(e+1) >> 24 (40 bits)."""
    return (2 * int(w) << 64) + 2 * (splitmix_output(seed, e + 1) >> 24)


@dataclass
class Result:
    edges: np.ndarray     # int32, ascending
    weight: int           # sum of the caller's weights over edges
    obs: int              # XOR of observable masks
    flags: int            # OF_* bits


class Graph:
    """Oracle handle on a detector graph (host copy + tie-broken weights)."""

    def __init__(self, g, tiebreak_seed: int):
        self.g = g
        self.seed = int(tiebreak_seed)
        self._h = _lib().oracle_graph_create(
            ctypes.c_int32(g.num_detectors), ctypes.c_int64(g.num_edges), _p(g.u), _p(g.v), _p(g.w),
            _p(g.obs_mask), ctypes.c_uint64(self.seed & ((1 << 64) - 1)))
        if not self._h:
            raise ValueError("oracle: invalid graph")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().oracle_graph_destroy(ctypes.c_void_p(h))
            self._h = None

    def tiebroken_weights(self):
        hi = np.zeros(self.g.num_edges, np.int64); lo = np.zeros(self.g.num_edges, np.uint64)
        _lib().oracle_tiebroken_weights(ctypes.c_void_p(self._h), _p(hi), _p(lo))
        return _join(hi, lo)

    def mwem(self, defects) -> Result:
        d = np.ascontiguousarray(defects, np.int32)
        cap = self.g.num_edges
        out = np.zeros(max(cap, 1), np.int32)
        n = ctypes.c_int64(); wt = ctypes.c_int64(); ob = ctypes.c_uint64()
        flags = _lib().oracle_mwem(ctypes.c_void_p(self._h), ctypes.c_int32(d.shape[0]), _p(d), _p(out),
                                   ctypes.c_int64(cap), ctypes.byref(n), ctypes.byref(wt), ctypes.byref(ob))
        return Result(out[: n.value].copy(), int(wt.value), int(ob.value), int(flags))

    def dijkstra(self, src: int):
        n = self.g.num_detectors
        hi = np.zeros(n, np.int64); lo = np.zeros(n, np.uint64); pred = np.zeros(n, np.int64)
        bh = ctypes.c_int64(); bl = ctypes.c_uint64(); be = ctypes.c_int64()
        _lib().oracle_dijkstra(ctypes.c_void_p(self._h), ctypes.c_int32(src), _p(hi), _p(lo), _p(pred),
                               ctypes.byref(bh), ctypes.byref(bl), ctypes.byref(be))
        bd = None if bh.value >= (1 << 62) else (int(bh.value) << 64) + int(bl.value)
        dist = [None if h >= (1 << 62) else (int(h) << 64) + int(l) for h, l in zip(hi.tolist(), lo.tolist())]
        return dist, pred, bd, int(be.value)

    def defect_distances(self, defects):
        d = np.ascontiguousarray(defects, np.int32)
        m = d.shape[0]
        hi = np.zeros(m * m, np.int64); lo = np.zeros(m * m, np.uint64)
        bh = np.zeros(m, np.int64); bl = np.zeros(m, np.uint64)
        _lib().oracle_defect_distances(ctypes.c_void_p(self._h), ctypes.c_int32(m), _p(d), _p(hi), _p(lo),
                                       _p(bh), _p(bl))
        D = _join(hi, lo)
        return [D[i * m:(i + 1) * m] for i in range(m)], _join(bh, bl)

    def boundary_table(self, defects):
        """Distances from each defect to the boundary vertex of every boundary edge."""
        d = np.ascontiguousarray(defects, np.int32)
        be = np.nonzero(self.g.v < 0)[0].astype(np.int64)
        m, nb = d.shape[0], be.shape[0]
        hi = np.zeros(m * nb, np.int64); lo = np.zeros(m * nb, np.uint64)
        _lib().oracle_defect_boundary_table(ctypes.c_void_p(self._h), ctypes.c_int32(m), _p(d),
                                            ctypes.c_int32(nb), _p(be), _p(hi), _p(lo))
        T = _join(hi, lo)
        return [T[i * nb:(i + 1) * nb] for i in range(m)]


SBF_INFEASIBLE, SBF_INTERNAL, SBF_DUAL, SBF_UNCLUSTERED, SBF_REACHED_LATER, SBF_CROSS_CLUSTER = 1, 2, 4, 8, 16, 32


@dataclass
class SBResult:
    edges: np.ndarray     # int32, ascending
    weight: int           # sum of the caller's weights over edges
    obs: int              # XOR of observable masks
    flags: int            # SBF_* bits
    levels: np.ndarray    # processing-cluster level of every detection event (1-based)
    events: int           # applied flooder/matcher events (ARRIVE, LEAVE, COLLIDE, IMPLODE, shatter)
    arrivals: int         # ARRIVE events
    e_ideal: int          # parallel event count (Methods, numerical evaluation)
    clusters: int         # processing clusters
    max_level: int        # highest level holding a cluster
    level1_search: int    # detectors inside the level-1 exploring regions, summed over events
    tied: int             # events applied while a different event was due at the same time (the counts of
                          # such shots can depend on the order of the simultaneous events; the result cannot)


class SparseBlossom:
    """Serial sparse blossom on a detector graph (``sparse_blossom.c``): global
    (every event in one cluster) or partition-and-fuse with a given level
    schedule.  Independent of ``Graph`` (mwem.c) and of the GPU path."""

    def __init__(self, g, tiebreak_seed: int):
        self.g = g
        self._h = _lib().oracle_sb_graph_create(
            ctypes.c_int32(g.num_detectors), ctypes.c_int64(g.num_edges), _p(np.ascontiguousarray(g.u, np.int32)),
            _p(np.ascontiguousarray(g.v, np.int32)), _p(np.ascontiguousarray(g.w, np.int32)),
            _p(np.ascontiguousarray(g.obs_mask, np.uint64)), ctypes.c_uint64(int(tiebreak_seed) & ((1 << 64) - 1)))
        if not self._h:
            raise ValueError("oracle: invalid graph")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().oracle_sb_graph_destroy(ctypes.c_void_p(h))
            self._h = None

    def decode(self, defects, d_sched=(), b_sched=(), reading: str = "strict", global_mode: bool = False) -> SBResult:
        """Decode one shot.  d_sched / b_sched: level parameters d_k, b_k
        (index 0 = level 1, exact ints in the tie-broken units), ignored in
        global mode."""
        d = np.ascontiguousarray(defects, np.int32)
        # levels whose parameters no longer fit the C side's 128-bit integers are never needed: every
        # graph here is accepted long before (the parameters grow geometrically)
        keep = [k for k in range(len(d_sched)) if max(int(d_sched[k]), int(b_sched[k])) < (1 << 123)]
        d_sched = [d_sched[k] for k in keep]; b_sched = [b_sched[k] for k in keep]
        nl = len(d_sched)
        mask = (1 << 64) - 1
        dh = np.asarray([int(x) >> 64 for x in d_sched] or [0], np.int64)
        dl = np.asarray([int(x) & mask for x in d_sched] or [0], np.uint64)
        bh = np.asarray([int(x) >> 64 for x in b_sched] or [0], np.int64)
        bl = np.asarray([int(x) & mask for x in b_sched] or [0], np.uint64)
        cap = max(self.g.num_edges, 1)
        out = np.zeros(cap, np.int32)
        lv = np.zeros(max(d.shape[0], 1), np.int8)
        st = np.zeros(8, np.int64)
        n = ctypes.c_int64(); wt = ctypes.c_int64(); ob = ctypes.c_uint64()
        _lib().oracle_sb_decode(ctypes.c_void_p(self._h), ctypes.c_int32(d.shape[0]), _p(d), ctypes.c_int32(nl),
                                _p(dh), _p(dl), _p(bh), _p(bl), ctypes.c_int32(1 if reading == "loose" else 0),
                                ctypes.c_int32(1 if global_mode else 0), _p(out), ctypes.c_int64(cap),
                                ctypes.byref(n), ctypes.byref(wt), ctypes.byref(ob), _p(lv), _p(st))
        return SBResult(out[: n.value].copy(), int(wt.value), int(ob.value), int(st[6]), lv[: d.shape[0]].copy(),
                        int(st[0]), int(st[1]), int(st[2]), int(st[3]), int(st[4]), int(st[5]), int(st[7]))


def max_weight_matching(W) -> tuple[list, bool]:
    """Maximum-weight matching of a dense non-negative integer weight matrix
    (0 = no edge) with the oracle's Edmonds implementation.  Returns (mate,
    certificate_ok)."""
    n = len(W)
    hi = np.zeros(n * n, np.int64); lo = np.zeros(n * n, np.uint64)
    for i in range(n):
        for j in range(n):
            x = int(W[i][j])
            hi[i * n + j] = x >> 64; lo[i * n + j] = x & ((1 << 64) - 1)
    mate = np.zeros(n, np.int32)
    ok = _lib().oracle_max_weight_matching(ctypes.c_int32(n), _p(hi), _p(lo), _p(mate))
    return mate.tolist(), bool(ok)


# ---------------------------------------------------------------------------
# Finite-size parameter schedule (Methods, Algorithm "Parameter schedule";
# Supplementary S11).
# ---------------------------------------------------------------------------

def phi_bar(k: int, q: Fraction, phi_min: Fraction) -> Fraction:
    """Target sequence  phi_bar_k = phi_min + (1 - phi_min) q^(k-1)."""
    return phi_min + (1 - phi_min) * q ** (k - 1)


def Phi_next(b, d_k, phi_k: Fraction) -> Fraction:
    """Phi_{k+1}(b) = phi_k - (phi_k + 2) d_k / ((phi_k + 1) d_k + phi_k b)."""
    return phi_k - (phi_k + 2) * d_k / ((phi_k + 1) * d_k + phi_k * b)


def _admissible(b, d_k, phi_k, target) -> bool:
    return b >= d_k and phi_k > Fraction(2 * d_k, b) and Phi_next(b, d_k, phi_k) >= target


def schedule(w_max: int, q: Fraction = Fraction(1, 10), phi_min: Fraction = Fraction(1, 100),
             levels: int = 6):
    """Return (d, b, phi) lists for levels 1..levels (index 0 = level 1).

    d_1 = w_max + 1, phi_1 = 1; b_k is the smallest integer with b_k >= d_k,
    phi_k > 2 d_k / b_k and Phi_{k+1}(b_k) >= phi_bar_{k+1};
    phi_{k+1} = Phi_{k+1}(b_k), d_{k+1} = 3 d_k + 4 b_k + 2 w_max.
    """
    q = Fraction(q); phi_min = Fraction(phi_min)
    d = [int(w_max) + 1]
    b = []
    phi = [Fraction(1)]
    for k in range(1, levels + 1):
        dk, pk = d[-1], phi[-1]
        target = phi_bar(k + 1, q, phi_min)
        # each condition is monotone in b; take the largest of the three lower bounds
        lo1 = dk
        lo2 = (2 * dk * pk.denominator) // pk.numerator + 1          # b > 2 d / phi
        gap = pk - target
        num = (pk + 2) * dk - gap * (pk + 1) * dk                     # phi * gap * b >= num
        lo3 = -((-num) // (pk * gap)) if num > 0 else 0               # ceil
        bk = max(lo1, lo2, int(lo3))
        while not _admissible(bk, dk, pk, target):                    # guard exactness
            bk += 1
        while bk - 1 >= 1 and _admissible(bk - 1, dk, pk, target):
            bk -= 1
        b.append(bk)
        phi.append(Phi_next(bk, dk, pk))
        d.append(3 * dk + 4 * bk + 2 * int(w_max))
    return d[:levels], b, phi[:levels]


# ---------------------------------------------------------------------------
# Processing-cluster hierarchy (Methods, Algorithm "Clustering").
# ---------------------------------------------------------------------------

def cluster_levels(D, BT, d_sched, b_sched, reading: str = "strict", components: bool = False):
    """Level of every defect under the clustering algorithm.

    D[i][j]   exact distance between defects i and j (None = unreachable);
    BT[i][k]  exact distance from defect i to the k-th boundary vertex;
    d_sched, b_sched: level parameters (index 0 = level 1).
    Exploring regions of radius b_k/2 around u and v touch iff D[u][v] <= b_k.
    A component is accepted iff its defect-set diameter is <= d_k and it has
    even size or reaches a boundary vertex: under reading "strict" some
    boundary vertex lies within d_k of every member; under "loose" some
    member's exploring region (radius b_k/2) reaches a boundary vertex.
    Returns a list of levels (1-based); 0 = never accepted within the schedule;
    with components=True also the accepted components (processing clusters)
    as (level, sorted member list) pairs.
    """
    m = len(D)
    level = [0] * m
    clusters = []
    residual = list(range(m))
    for k in range(len(d_sched)):
        if not residual:
            break
        dk, bk = d_sched[k], b_sched[k]
        seen = set()
        comps = []
        for s in residual:
            if s in seen:
                continue
            comp, stack = [], [s]
            seen.add(s)
            while stack:
                x = stack.pop(); comp.append(x)
                for y in residual:
                    if y not in seen and D[x][y] is not None and D[x][y] <= bk:
                        seen.add(y); stack.append(y)
            comps.append(sorted(comp))
        accepted = []
        for comp in comps:
            diam_ok = all(D[x][y] is not None and D[x][y] <= dk for x in comp for y in comp)
            if not diam_ok:
                continue
            if len(comp) % 2 == 0:
                ok = True
            elif reading == "strict":
                nb = len(BT[comp[0]]) if comp else 0
                ok = any(all(BT[x][j] is not None and BT[x][j] <= dk for x in comp) for j in range(nb))
            else:
                ok = any(2 * BT[x][j] <= bk for x in comp for j in range(len(BT[x])) if BT[x][j] is not None)
            if ok:
                accepted.append(comp)
        for comp in accepted:
            clusters.append((k + 1, comp))
            for x in comp:
                level[x] = k + 1
        acc = {x for c in accepted for x in c}
        residual = [x for x in residual if x not in acc]
    return (level, clusters) if components else level


# ---------------------------------------------------------------------------
# Brute-force pins for tiny inputs.
# ---------------------------------------------------------------------------

def brute_mwem_edges(g, defects, seed: int):
    """Enumerate every edge subset (|E| <= 22) and return the tie-broken
    minimum-weight subset whose odd-degree detectors are exactly `defects`."""
    E = g.num_edges
    assert E <= 22
    # keyed on the graph's content: an id() can be reused by a later graph
    key = (g.u.tobytes(), g.v.tobytes(), np.asarray(g.w).tobytes(), int(seed))
    if key not in _brute_cache:
        masks = np.arange(1 << E, dtype=np.int64)
        bits = ((masks[:, None] >> np.arange(E)[None, :]) & 1).astype(np.int64)   # [2^E, E]
        # odd-degree signature of every subset, packed as an integer bitmask of detectors
        sig = np.zeros(1 << E, np.int64)
        for e in range(E):
            for x in (int(g.u[e]), int(g.v[e])):
                if x >= 0:
                    sig ^= bits[:, e] << x
        prim = bits @ np.asarray([2 * int(g.w[e]) for e in range(E)], np.int64)
        sec = bits @ np.asarray([2 * (splitmix_output(seed, e + 1) >> 24) for e in range(E)], np.int64)
        _brute_cache.clear()
        _brute_cache[key] = (sig, prim, sec)
    sig, prim, sec = _brute_cache[key]
    target = 0
    for x in defects:
        target |= 1 << int(x)
    idx = np.nonzero(sig == target)[0]
    if idx.size == 0:
        return None
    # lexicographic (primary, secondary) = exact order of wt = primary*2^64 + secondary
    order = np.lexsort((sec[idx], prim[idx]))
    best = int(idx[order[0]])
    return [e for e in range(E) if best >> e & 1]


_brute_cache: dict = {}


def brute_min_pairing(costs_pair, costs_bd):
    """Minimum-cost pairing of m items where each item is paired with another
    item (costs_pair[i][j], None = forbidden) or with the boundary
    (costs_bd[i], None = forbidden); exhaustive recursion (m <= 10)."""
    m = len(costs_bd)

    def rec(rest):
        if not rest:
            return 0
        i = rest[0]
        best = None
        if costs_bd[i] is not None:
            r = rec(rest[1:])
            if r is not None:
                best = costs_bd[i] + r
        for j in rest[1:]:
            c = costs_pair[i][j]
            if c is None:
                continue
            r = rec([x for x in rest[1:] if x != j])
            if r is not None and (best is None or c + r < best):
                best = c + r
        return best

    return rec(list(range(m)))


# ---------------------------------------------------------------------------
# Sliding-window decoding (Introduction: long streams of rounds decoded in
# overlapping windows).  Parity unpinned beyond its own properties: the paper
# fixes no window rule; this is the plain procedure the decoder implements.
# ---------------------------------------------------------------------------

@dataclass
class WindowGraph:
    num_detectors: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    obs_mask: np.ndarray

    @property
    def num_edges(self) -> int:
        return int(self.u.shape[0])


def window_schedule(g, layer_size: int, window_layers: int, commit_layers: int):
    """Windows of `window_layers` layers advancing by `commit_layers`: list of
    (first layer, window graph, full-graph edge id of each window edge, commit
    flag of each window edge).  Inside window [a, b): an edge with both ends in
    it is kept; an edge from it to a later layer ends at the boundary; an edge
    to an earlier layer is left out.  A matched edge is committed when its
    lower layer is below a + commit_layers, or in the last window (which
    reaches the final layer)."""
    L = int(layer_size)
    n_layers = g.num_detectors // L
    out = []
    a = 0
    while True:
        last = a + window_layers >= n_layers
        b = n_layers if last else a + window_layers
        wu, wv, ww, wo, emap, commit = [], [], [], [], [], []
        for e in range(g.num_edges):
            x, y = int(g.u[e]), int(g.v[e])
            lx = x // L
            if y < 0:
                if not (a <= lx < b):
                    continue
                ends, low = (x - a * L, -1), lx
            else:
                ly = y // L
                inx, iny = a <= lx < b, a <= ly < b
                if inx and iny:
                    ends, low = (x - a * L, y - a * L), min(lx, ly)
                elif inx and ly >= b:
                    ends, low = (x - a * L, -1), lx
                elif iny and lx >= b:
                    ends, low = (y - a * L, -1), ly
                else:
                    continue
            wu.append(ends[0]); wv.append(ends[1]); ww.append(int(g.w[e])); wo.append(int(g.obs_mask[e]))
            emap.append(e)
            commit.append(last or low < a + commit_layers)
        wg = WindowGraph((b - a) * L, np.asarray(wu, np.int32), np.asarray(wv, np.int32),
                         np.asarray(ww, np.int32), np.asarray(wo, np.uint64))
        out.append((a, wg, emap, commit))
        if last:
            return out
        a += commit_layers


def window_decode(g, schedule, graphs, layer_size: int, defects):
    """Decode one shot window by window.  `graphs[k]` is an oracle ``Graph`` on
    the k-th window graph of `schedule`.  Returns (weight, obs, ok): the sum of
    the committed edges' weights, the XOR of their observable masks, and
    whether every detection event ended resolved and every window was
    feasible."""
    L = int(layer_size)
    running = set(int(x) for x in defects)
    weight, obs = 0, 0
    for (a, wg, emap, commit), og in zip(schedule, graphs):
        lo, hi = a * L, a * L + wg.num_detectors
        local = sorted(x - lo for x in running if lo <= x < hi)
        r = og.mwem(np.asarray(local, np.int32))
        if r.flags & OF_INFEASIBLE:
            return 0, 0, False
        for e in r.edges.tolist():
            if not commit[e]:
                continue
            ge = emap[e]
            weight += int(g.w[ge])
            obs ^= int(g.obs_mask[ge])
            for end in (int(g.u[ge]), int(g.v[ge])):
                if end >= 0:
                    running ^= {end}
    return weight, obs, not running


# ---------------------------------------------------------------------------
# Complementary gap (Introduction: the gap between the best correction and the
# best one with the other value of a logical observable).
# ---------------------------------------------------------------------------

class Complementary:
    """The two constrained minima for observable bit `obs_bit`, whose edges
    must all be boundary edges.  Each observable edge j is rerouted to a new
    detector x_j, consecutive x_j are joined by weight-1 edges, and the
    original weights are scaled by S (a power of two at least the number of
    observable edges): an edge set with odd degree exactly at D (and at x_1
    when asked) has observable parity equal to the number of active x_j, and
    its chain part weighs less than S."""

    def __init__(self, g, obs_bit: int, tiebreak_seed: int):
        bit = 1 << int(obs_bit)
        cut = [e for e in range(g.num_edges) if int(g.obs_mask[e]) & bit]
        if not cut or any(int(g.v[e]) >= 0 for e in cut):
            raise ValueError("the observable must be carried by boundary edges only")
        S = 1
        while S < len(cut):
            S *= 2
        n = g.num_detectors
        u = [int(x) for x in g.u]; v = [int(x) for x in g.v]
        w = [int(x) * S for x in g.w]; ob = [int(x) for x in g.obs_mask]
        for j, e in enumerate(cut):
            v[e] = n + j
        for j in range(len(cut) - 1):
            u.append(n + j); v.append(n + j + 1); w.append(1); ob.append(0)
        self.n, self.S, self.bit = n, S, bit
        self.graph = WindowGraph(n + len(cut), np.asarray(u, np.int32), np.asarray(v, np.int32),
                                 np.asarray(w, np.int32), np.asarray(ob, np.uint64))
        self.og = Graph(self.graph, tiebreak_seed)

    def weights(self, defects):
        """(W0, W1): minimum original weight with the observable bit 0 and 1
        (None where no such edge set exists)."""
        d = sorted(int(x) for x in defects)
        out = []
        for extra in ([], [self.n]):
            r = self.og.mwem(np.asarray(d + extra, np.int32))
            out.append(None if r.flags & OF_INFEASIBLE else r.weight // self.S)
        return tuple(out)
