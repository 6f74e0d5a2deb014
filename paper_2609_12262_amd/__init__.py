"""Thin Python binding of libpsb (parallel sparse-blossom decoding on MI355X).

Argument marshalling only: every step of decoding runs in the HIP library.
PyTorch provides device memory and the current stream.  The names follow the
C ABI in include/psb.h.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsb.so")

PSB_OK = 0
PSB_S_OK, PSB_S_CAPACITY, PSB_S_INFEASIBLE, PSB_S_EDGES_TRUNCATED, PSB_S_INTERNAL = 0, 1, 2, 3, 4
PSB_S_CANCELLED = 6
PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED, PSB_E_INTERNAL = -1, -2, -3, -4, -5
MODE_PARTITION, MODE_GLOBAL = 0, 1

_lib = None


class PsbError(RuntimeError):
    pass


class _GraphDesc(ctypes.Structure):
    _fields_ = [("num_detectors", ctypes.c_int32), ("num_edges", ctypes.c_int64),
                ("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("obs_mask", ctypes.c_void_p)]


class _DecoderOpts(ctypes.Structure):
    _fields_ = [("q_num", ctypes.c_int64), ("q_den", ctypes.c_int64),
                ("phi_min_num", ctypes.c_int64), ("phi_min_den", ctypes.c_int64),
                ("tiebreak_seed", ctypes.c_uint64), ("mode", ctypes.c_int32),
                ("boundary_reading", ctypes.c_int32), ("max_defects_per_shot", ctypes.c_int32),
                ("edges_per_shot", ctypes.c_int32), ("num_slots", ctypes.c_int32),
                ("fast_max_nodes", ctypes.c_int32), ("fast_max_regions", ctypes.c_int32),
                ("overflow_slots", ctypes.c_int32), ("first_tier", ctypes.c_int32),
                ("fast_lds_state", ctypes.c_int32), ("event_accounting", ctypes.c_int32),
                ("serial_level_one", ctypes.c_int32), ("cluster_walk", ctypes.c_int32)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("opts", _DecoderOpts), ("ms", ctypes.c_float), ("status", ctypes.c_int32)]


def _make_opts(tiebreak_seed: int = 0x5EED, mode: int = 0, boundary_reading: int = 0, max_defects: int = 0,
               edges_per_shot: int = 0, num_slots: int = 0, q=(1, 10), phi_min=(1, 100), fast_max_nodes: int = 0,
               fast_max_regions: int = 0, overflow_slots: int = 0, first_tier: int = 0,
               fast_lds_state: int = 0, event_accounting: int = 0, serial_level_one: int = 0,
               cluster_walk: int = 0) -> _DecoderOpts:
    return _DecoderOpts(q[0], q[1], phi_min[0], phi_min[1], tiebreak_seed & ((1 << 64) - 1), mode,
                        boundary_reading, max_defects, edges_per_shot, num_slots, fast_max_nodes,
                        fast_max_regions, overflow_slots, first_tier, fast_lds_state, event_accounting,
                        serial_level_one, cluster_walk)


def _opts_kwargs(o: _DecoderOpts) -> dict:
    """Decoder keyword arguments equal to an options record."""
    return {"tiebreak_seed": o.tiebreak_seed, "mode": o.mode, "boundary_reading": o.boundary_reading,
            "max_defects": o.max_defects_per_shot, "edges_per_shot": o.edges_per_shot, "num_slots": o.num_slots,
            "q": (o.q_num, o.q_den), "phi_min": (o.phi_min_num, o.phi_min_den),
            "fast_max_nodes": o.fast_max_nodes, "fast_max_regions": o.fast_max_regions,
            "overflow_slots": o.overflow_slots, "first_tier": o.first_tier, "fast_lds_state": o.fast_lds_state,
            "event_accounting": o.event_accounting, "serial_level_one": o.serial_level_one,
            "cluster_walk": o.cluster_walk}


def lib():
    """The loaded libpsb.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PsbError(f"{LIB_PATH} is missing: build it with paper_2609_12262_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.psb_last_error.restype = ctypes.c_char_p
        for name in ("psb_graph_create", "psb_graph_destroy", "psb_decoder_create", "psb_decoder_destroy",
                     "psb_decode_batch", "psb_decode_batch_noalloc", "psb_decoder_levels", "psb_decoder_edges_per_shot",
                     "psb_decoder_max_defects", "psb_graph_syndrome_bytes", "psb_schedule_levels",
                     "psb_decoder_slots", "psb_decoder_last_overflow", "psb_decoder_device_bytes", "psb_decoder_reserve",
                     "psb_server_create", "psb_server_submit", "psb_server_submit_many", "psb_server_poll", "psb_server_collect",
                     "psb_server_stats", "psb_server_destroy", "psb_server_cancel", "psb_server_wait", "psb_autotune", "psb_autotune_candidates",
                     "psb_batch_graph_create", "psb_batch_graph_launch", "psb_batch_graph_destroy",
                     "psb_window_plan_create", "psb_window_plan_info", "psb_window_decode",
                     "psb_window_plan_destroy", "psb_comp_plan_create", "psb_comp_decode",
                     "psb_comp_plan_destroy", "psb_slot_server_create", "psb_slot_server_submit_many",
                     "psb_slot_server_collect", "psb_slot_server_collect_edges", "psb_slot_server_poll",
                     "psb_slot_server_stats", "psb_slot_server_destroy", "psb_stream_server_create", "psb_stream_push", "psb_stream_push_many",
                     "psb_stream_poll", "psb_stream_latencies", "psb_stream_reset", "psb_stream_server_info",
                     "psb_stream_server_destroy"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc < 0:
        raise PsbError(f"{what}: {lib().psb_last_error().decode()} (code {rc})")
    return rc


def schedule_levels(w_max: int, diam: int, q=(1, 10), phi_min=(1, 100), max_levels: int = 16):
    """Level parameters (d_k, b_k, final) from the library's host-side schedule."""
    M = (1 << 64) - 1
    arr = [np.zeros(max_levels, np.uint64) for _ in range(4)]
    fin = np.zeros(max_levels, np.int32)
    n = _check(lib().psb_schedule_levels(
        ctypes.c_uint64(w_max >> 64), ctypes.c_uint64(w_max & M), ctypes.c_uint64(diam >> 64),
        ctypes.c_uint64(diam & M), ctypes.c_int64(q[0]), ctypes.c_int64(q[1]), ctypes.c_int64(phi_min[0]),
        ctypes.c_int64(phi_min[1]), ctypes.c_int32(max_levels), *[ctypes.c_void_p(a.ctypes.data) for a in arr],
        ctypes.c_void_p(fin.ctypes.data)), "psb_schedule_levels")
    d = [(int(arr[0][k]) << 64) | int(arr[1][k]) for k in range(n)]
    b = [(int(arr[2][k]) << 64) | int(arr[3][k]) for k in range(n)]
    return d, b, fin[:n].tolist()


class Graph:
    """Device-resident detector graph (psb_graph_create)."""

    def __init__(self, num_detectors: int, u, v, w, obs_mask):
        self.u = np.ascontiguousarray(u, np.int32)
        self.v = np.ascontiguousarray(v, np.int32)
        self.w = np.ascontiguousarray(w, np.int32)
        self.obs_mask = np.ascontiguousarray(obs_mask, np.uint64)
        self.num_detectors = int(num_detectors)
        desc = _GraphDesc(self.num_detectors, self.u.shape[0], self.u.ctypes.data, self.v.ctypes.data,
                          self.w.ctypes.data, self.obs_mask.ctypes.data)
        h = ctypes.c_void_p()
        _check(lib().psb_graph_create(ctypes.byref(desc), ctypes.byref(h)), "psb_graph_create")
        self._h = h

    @classmethod
    def from_synth(cls, g):
        return cls(g.num_detectors, g.u, g.v, g.w, g.obs_mask)

    @property
    def syndrome_bytes(self) -> int:
        return lib().psb_graph_syndrome_bytes(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Batch:
    edges: "object"      # torch int32 [n, edges_per_shot] (device)
    n_edges: "object"    # torch int32 [n]
    weight: "object"     # torch int64 [n]
    obs: "object"        # torch uint64 as int64 view [n]
    status: "object"     # torch int32 [n]
    levels: "object"     # torch int8 [n, max_defects] or None
    t_done: "object"     # torch int64 [n+1] (device clock ticks; [n] = launch start) or None
    stats: "object"      # torch int32 [n, 8] or None


class Decoder:
    """psb_decoder: schedule, tie-break weights and device workspaces."""

    def __init__(self, graph: Graph, tiebreak_seed: int = 0x5EED, mode: int = MODE_PARTITION,
                 boundary_reading: int = 0, max_defects: int = 0, edges_per_shot: int = 0,
                 num_slots: int = 0, q=(1, 10), phi_min=(1, 100), fast_max_nodes: int = 0,
                 fast_max_regions: int = 0, overflow_slots: int = 0, first_tier: int = 0, fast_lds_state: int = 0,
                 event_accounting: int = 0, serial_level_one: int = 0, cluster_walk: int = 0):
        self.graph = graph
        opts = _make_opts(tiebreak_seed, mode, boundary_reading, max_defects, edges_per_shot, num_slots, q, phi_min,
                          fast_max_nodes, fast_max_regions, overflow_slots, first_tier, fast_lds_state,
                          event_accounting, serial_level_one, cluster_walk)
        self.stats_width = 12 if event_accounting else 8
        h = ctypes.c_void_p()
        _check(lib().psb_decoder_create(graph._h, ctypes.byref(opts), ctypes.byref(h)), "psb_decoder_create")
        self._h = h
        self.edges_per_shot = lib().psb_decoder_edges_per_shot(h)
        self.max_defects = lib().psb_decoder_max_defects(h)
        fs, os_, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().psb_decoder_slots(h, ctypes.byref(fs), ctypes.byref(os_), ctypes.byref(lds)), "psb_decoder_slots")
        self.fast_slots, self.overflow_slots, self.fast_lds_bytes = fs.value, os_.value, lds.value

    def levels(self, max_levels: int = 16):
        arr = [np.zeros(max_levels, t) for t in (np.int64, np.uint64, np.int64, np.uint64)]
        fin = np.zeros(max_levels, np.int32)
        n = _check(lib().psb_decoder_levels(self._h, ctypes.c_int32(max_levels),
                                            *[ctypes.c_void_p(a.ctypes.data) for a in arr],
                                            ctypes.c_void_p(fin.ctypes.data)), "psb_decoder_levels")
        d = [(int(arr[0][k]) << 64) + int(arr[1][k]) for k in range(n)]
        b = [(int(arr[2][k]) << 64) + int(arr[3][k]) for k in range(n)]
        return d, b, fin[:n].tolist()

    def alloc(self, n: int, levels: bool = False, timestamps: bool = False, stats: bool = False,
              device="cuda") -> Batch:
        import torch
        return Batch(
            edges=torch.empty((n, self.edges_per_shot), dtype=torch.int32, device=device),
            n_edges=torch.empty(n, dtype=torch.int32, device=device),
            weight=torch.empty(n, dtype=torch.int64, device=device),
            obs=torch.empty(n, dtype=torch.int64, device=device),
            status=torch.empty(n, dtype=torch.int32, device=device),
            levels=torch.zeros((n, self.max_defects), dtype=torch.int8, device=device) if levels else None,
            t_done=torch.zeros(n + 1, dtype=torch.int64, device=device) if timestamps else None,
            stats=torch.zeros((n, self.stats_width), dtype=torch.int32, device=device) if stats else None)

    def decode_into(self, syndromes, out: Batch, stream=None) -> Batch:
        """Launch psb_decode_batch on `stream` (default: torch's current stream)."""
        import torch
        if not syndromes.is_cuda or syndromes.dtype != torch.uint8 or not syndromes.is_contiguous():
            raise PsbError("syndromes must be a contiguous uint8 CUDA tensor")
        n = syndromes.shape[0]
        if n and syndromes.shape[1] != self.graph.syndrome_bytes:
            raise PsbError(f"syndrome rows must have {self.graph.syndrome_bytes} bytes")
        if out.edges.shape[0] < n:
            raise PsbError("output batch too small")
        s = stream if stream is not None else torch.cuda.current_stream()
        P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
        _check(lib().psb_decode_batch(self._h, P(syndromes), ctypes.c_int64(n), P(out.edges), P(out.n_edges),
                                      P(out.weight), P(out.obs), P(out.status), P(out.levels), P(out.t_done),
                                      P(out.stats), ctypes.c_void_p(s.cuda_stream)), "psb_decode_batch")
        return out

    def decode_into_noalloc(self, syndromes, out: Batch, stream=None) -> Batch:
        """psb_decode_batch_noalloc on `stream`: the same decode with no device allocation in the call
        (counters and overflow list in the library's fixed per-device array; at most PSB_NOALLOC_MAX_SHOTS)."""
        import torch
        if not syndromes.is_cuda or syndromes.dtype != torch.uint8 or not syndromes.is_contiguous():
            raise PsbError("syndromes must be a contiguous uint8 CUDA tensor")
        n = syndromes.shape[0]
        if n and syndromes.shape[1] != self.graph.syndrome_bytes:
            raise PsbError(f"syndrome rows must have {self.graph.syndrome_bytes} bytes")
        if out.edges.shape[0] < n:
            raise PsbError("output batch too small")
        s = stream if stream is not None else torch.cuda.current_stream()
        P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
        _check(lib().psb_decode_batch_noalloc(self._h, P(syndromes), ctypes.c_int64(n), P(out.edges),
                                              P(out.n_edges), P(out.weight), P(out.obs), P(out.status),
                                              P(out.levels), P(out.t_done), P(out.stats),
                                              ctypes.c_void_p(s.cuda_stream)), "psb_decode_batch_noalloc")
        return out

    def decode(self, syndromes, levels: bool = False, timestamps: bool = False, stats: bool = False) -> Batch:
        out = self.alloc(syndromes.shape[0], levels, timestamps, stats, device=syndromes.device)
        return self.decode_into(syndromes, out)

    def capture(self, syndromes, out: Batch) -> "BatchGraph":
        """Capture psb_decode_batch(syndromes -> out) into a HIP graph; refill `syndromes` in place and
        replay with BatchGraph.launch()."""
        import torch
        if not syndromes.is_cuda or syndromes.dtype != torch.uint8 or not syndromes.is_contiguous():
            raise PsbError("syndromes must be a contiguous uint8 CUDA tensor")
        n = syndromes.shape[0]
        if out.edges.shape[0] < n:
            raise PsbError("output batch too small")
        P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
        h = ctypes.c_void_p()
        _check(lib().psb_batch_graph_create(self._h, P(syndromes), ctypes.c_int64(n), P(out.edges), P(out.n_edges),
                                            P(out.weight), P(out.obs), P(out.status), P(out.levels),
                                            P(out.t_done), P(out.stats), ctypes.byref(h)), "psb_batch_graph_create")
        return BatchGraph(h, (self, syndromes, out))

    def reserve(self, max_batch: int):
        """Pre-size per-batch storage so that batches up to max_batch never reallocate."""
        _check(lib().psb_decoder_reserve(self._h, ctypes.c_int64(int(max_batch))), "psb_decoder_reserve")

    def last_overflow(self, stream=None) -> int:
        """Shots of the last batch decoded by the overflow tier (synchronises)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        n = ctypes.c_int32()
        _check(lib().psb_decoder_last_overflow(self._h, ctypes.c_void_p(s.cuda_stream), ctypes.byref(n)),
               "psb_decoder_last_overflow")
        return n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_decoder_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """psb_batch_graph: one captured psb_decode_batch call, replayed with a single graph launch."""

    def __init__(self, h, keep):
        self._h = h
        self._keep = keep            # decoder and buffers the graph's arguments point into

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().psb_batch_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream)), "psb_batch_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WindowPlan:
    """psb_window_plan: sliding-window decoding of a layered graph (one layer of detectors per round)."""

    def __init__(self, g, layer_size: int, window_layers: int, commit_layers: int, **opts):
        u = np.ascontiguousarray(g.u, np.int32); v = np.ascontiguousarray(g.v, np.int32)
        w = np.ascontiguousarray(g.w, np.int32); o = np.ascontiguousarray(g.obs_mask, np.uint64)
        desc = _GraphDesc(g.num_detectors, len(u), u.ctypes.data, v.ctypes.data, w.ctypes.data, o.ctypes.data)
        c = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().psb_window_plan_create(ctypes.byref(desc), ctypes.c_int32(layer_size),
                                            ctypes.c_int32(window_layers), ctypes.c_int32(commit_layers),
                                            ctypes.byref(c), ctypes.byref(h)), "psb_window_plan_create")
        self._h = h
        nw, ns = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().psb_window_plan_info(h, ctypes.byref(nw), ctypes.byref(ns)), "psb_window_plan_info")
        self.n_windows, self.n_shapes = nw.value, ns.value

    def decode(self, syndromes, stream=None):
        """syndromes: uint8 CUDA tensor [n][ceil(num_detectors/8)] -> dict of weight, obs, status tensors."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        n = syndromes.shape[0]
        out = dict(weight=torch.empty(n, dtype=torch.int64, device=syndromes.device),
                   obs=torch.empty(n, dtype=torch.int64, device=syndromes.device),
                   status=torch.empty(n, dtype=torch.int32, device=syndromes.device))
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check(lib().psb_window_decode(self._h, P(syndromes), ctypes.c_int64(n), P(out["weight"]), P(out["obs"]),
                                       P(out["status"]), ctypes.c_void_p(s.cuda_stream)), "psb_window_decode")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_window_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ComplementaryPlan:
    """psb_comp_plan: minimum weights under each value of one observable bit, and their gap."""

    def __init__(self, g, obs_bit: int = 0, **opts):
        u = np.ascontiguousarray(g.u, np.int32); v = np.ascontiguousarray(g.v, np.int32)
        w = np.ascontiguousarray(g.w, np.int32); o = np.ascontiguousarray(g.obs_mask, np.uint64)
        desc = _GraphDesc(g.num_detectors, len(u), u.ctypes.data, v.ctypes.data, w.ctypes.data, o.ctypes.data)
        c = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().psb_comp_plan_create(ctypes.byref(desc), ctypes.c_int32(obs_bit), ctypes.byref(c),
                                          ctypes.byref(h)), "psb_comp_plan_create")
        self._h = h

    def decode(self, syndromes, stream=None):
        """syndromes: uint8 CUDA tensor [n][ceil(num_detectors/8)] -> dict of weight0, weight1, gap, obs, status."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        n = syndromes.shape[0]
        dev = syndromes.device
        out = {k: torch.empty(n, dtype=torch.int64, device=dev) for k in ("weight0", "weight1", "gap", "obs")}
        out["status"] = torch.empty(n, dtype=torch.int32, device=dev)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check(lib().psb_comp_decode(self._h, P(syndromes), ctypes.c_int64(n), P(out["weight0"]), P(out["weight1"]),
                                     P(out["gap"]), P(out["obs"]), P(out["status"]), ctypes.c_void_p(s.cuda_stream)),
               "psb_comp_decode")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_comp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(graph: "Graph", syndromes, reps: int = 2, stream=None, **base):
    """Times every candidate configuration on the sample batch `syndromes` (uint8 device tensor) and
    returns (keyword arguments of the fastest Decoder, list of per-candidate records)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    nc = lib().psb_autotune_candidates()
    entries = (_TuneEntry * nc)()
    best = ctypes.c_int32(-1)
    b = _make_opts(**base)
    _check(lib().psb_autotune(graph._h, ctypes.byref(b), ctypes.c_void_p(syndromes.data_ptr()),
                              ctypes.c_int64(syndromes.shape[0]), ctypes.c_int32(reps),
                              ctypes.c_void_p(s.cuda_stream), entries, ctypes.c_int32(nc), ctypes.byref(best)),
           "psb_autotune")
    table = [dict(_opts_kwargs(e.opts), ms=round(float(e.ms), 4), status=int(e.status)) for e in entries]
    return _opts_kwargs(entries[best.value].opts), table


class Server:
    """psb_server: windows submitted one at a time while earlier ones decode."""

    def __init__(self, graphs, opts=None, device_mem_budget: int = 0, stream=None):
        """opts: None, one dict of Decoder keyword arguments for every graph, or a list of them (one per graph)."""
        self.graphs = list(graphs)
        per = opts if isinstance(opts, (list, tuple)) else [opts] * len(self.graphs)
        if len(per) != len(self.graphs):
            raise PsbError("one options record per graph")
        c = (_DecoderOpts * len(self.graphs))(*[_make_opts(**(o or {})) for o in per])
        arr = (ctypes.c_void_p * len(self.graphs))(*[g._h.value for g in self.graphs])
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p(0)
        _check(lib().psb_server_create(arr, ctypes.c_int32(len(self.graphs)), c,
                                       ctypes.c_int64(device_mem_budget), s, ctypes.byref(h)), "psb_server_create")
        self._h = h

    def submit(self, graph_idx: int, syndrome, w_override=None) -> int:
        syn = np.ascontiguousarray(syndrome, np.uint8)
        t = ctypes.c_uint64()
        wp = ctypes.c_void_p(0)
        if w_override is not None:
            w_override = np.ascontiguousarray(w_override, np.int32)
            wp = ctypes.c_void_p(w_override.ctypes.data)
        _check(lib().psb_server_submit(self._h, ctypes.c_int32(graph_idx), ctypes.c_void_p(syn.ctypes.data), wp,
                                       ctypes.byref(t)), "psb_server_submit")
        return t.value

    def submit_many(self, graph_idx, syndromes, uniform_weight=None) -> list:
        """Queue several windows in one call; uniform_weight[i] = 0 keeps the graph's weights."""
        n = len(syndromes)
        rows = [np.ascontiguousarray(r, np.uint8) for r in syndromes]
        ptrs = (ctypes.c_void_p * n)(*[r.ctypes.data for r in rows])
        gi = np.ascontiguousarray(graph_idx, np.int32)
        uw = None if uniform_weight is None else np.ascontiguousarray(uniform_weight, np.int32)
        t = np.zeros(n, np.uint64)
        _check(lib().psb_server_submit_many(self._h, ctypes.c_int32(n), ctypes.c_void_p(gi.ctypes.data), ptrs,
                                            ctypes.c_void_p(uw.ctypes.data) if uw is not None else ctypes.c_void_p(0),
                                            ctypes.c_void_p(t.ctypes.data)), "psb_server_submit_many")
        return [int(x) for x in t]

    def poll(self, ticket: int, edges_cap: int = 1024):
        """None while pending, else dict(weight, obs, edges, status, latency_ns)."""
        done = ctypes.c_int32(); w = ctypes.c_int64(); ob = ctypes.c_uint64(); ne = ctypes.c_int64()
        st = ctypes.c_int32(); lat = ctypes.c_int64()
        edges = np.zeros(max(edges_cap, 1), np.int32)
        _check(lib().psb_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(w),
                                     ctypes.byref(ob), ctypes.c_void_p(edges.ctypes.data), ctypes.c_int64(edges_cap),
                                     ctypes.byref(ne), ctypes.byref(st), ctypes.byref(lat)), "psb_server_poll")
        if not done.value:
            return None
        return dict(weight=w.value, obs=ob.value, edges=edges[: min(ne.value, edges_cap)].copy(), n_edges=ne.value,
                    status=st.value, latency_ns=lat.value)

    def cancel(self, ticket: int) -> bool:
        """psb_server_cancel: True if the window was still waiting and is now cancelled."""
        c = ctypes.c_int32()
        _check(lib().psb_server_cancel(self._h, ctypes.c_uint64(ticket), ctypes.byref(c)), "psb_server_cancel")
        return bool(c.value)

    def wait(self, ticket: int, timeout_us: int) -> bool:
        """psb_server_wait: True once the window is done, False on time-out."""
        d = ctypes.c_int32()
        _check(lib().psb_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.c_int64(int(timeout_us)),
                                     ctypes.byref(d)), "psb_server_wait")
        return bool(d.value)

    def collect(self, max_n: int = 4096) -> list:
        """Finished windows in completion order (without edge lists): dicts of ticket, weight, obs, status,
        latency_ns; empty when none is finished."""
        t = np.zeros(max(max_n, 1), np.uint64); w = np.zeros_like(t, dtype=np.int64)
        ob = np.zeros_like(t); st = np.zeros(len(t), np.int32); lat = np.zeros(len(t), np.int64)
        P = lambda a: ctypes.c_void_p(a.ctypes.data)
        k = _check(lib().psb_server_collect(self._h, ctypes.c_int32(max_n), P(t), P(w), P(ob), P(st), P(lat)),
                   "psb_server_collect")
        return [dict(ticket=int(t[i]), weight=int(w[i]), obs=int(ob[i]), status=int(st[i]), latency_ns=int(lat[i]))
                for i in range(k)]

    def stats(self) -> dict:
        """Running totals: batches, windows, mean submit-to-launch and launch-to-completion times."""
        v = (ctypes.c_int64 * 5)()
        _check(lib().psb_server_stats(self._h, v), "psb_server_stats")
        b, w = max(v[0], 1), max(v[1], 1)
        return {"batches": v[0], "windows": v[1], "mean_batch": v[1] / b, "mean_queue_us": v[2] / w / 1e3,
                "mean_batch_run_us": v[3] / b / 1e3, "mean_launch_us": v[4] / b / 1e3}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlotServer:
    """psb_slot_server: slot-level serving.  One persistent kernel whose wavefronts take windows one at a time
    as they are published; each window starts as soon as a slot is free and completes on its own.  While it
    runs, a device-wide synchronisation (torch.cuda.synchronize()) would wait for it: close it first."""

    def __init__(self, graphs, opts=None, waves: int = 0, ring: int = 0):
        self.graphs = list(graphs)
        per = opts if isinstance(opts, (list, tuple)) else [opts] * len(self.graphs)
        arr = (ctypes.c_void_p * len(self.graphs))(*[g._h.value for g in self.graphs])
        c = (_DecoderOpts * len(self.graphs))(*[_make_opts(**(o or {})) for o in per])
        h = ctypes.c_void_p()
        _check(lib().psb_slot_server_create(arr, ctypes.c_int32(len(self.graphs)), c, ctypes.c_int32(waves),
                                            ctypes.c_int32(ring), ctypes.byref(h)), "psb_slot_server_create")
        self._h = h

    def submit_many(self, graph_idx, syndromes, uniform_weight=None) -> list:
        n = len(syndromes)
        rows = [np.ascontiguousarray(r, np.uint8) for r in syndromes]
        ptrs = (ctypes.c_void_p * n)(*[r.ctypes.data for r in rows])
        gi = np.ascontiguousarray(graph_idx, np.int32)
        uw = None if uniform_weight is None else np.ascontiguousarray(uniform_weight, np.int32)
        t = np.zeros(n, np.uint64)
        _check(lib().psb_slot_server_submit_many(self._h, ctypes.c_int32(n), ctypes.c_void_p(gi.ctypes.data), ptrs,
                                                 ctypes.c_void_p(uw.ctypes.data) if uw is not None else ctypes.c_void_p(0),
                                                 ctypes.c_void_p(t.ctypes.data)), "psb_slot_server_submit_many")
        return [int(x) for x in t]

    def poll(self, ticket: int, edges_cap: int = 1024):
        """None while pending, else dict(weight, obs, edges, n_edges, status, latency_ns)."""
        done = ctypes.c_int32(); w = ctypes.c_int64(); ob = ctypes.c_uint64(); ne = ctypes.c_int64()
        st = ctypes.c_int32(); lat = ctypes.c_int64()
        edges = np.zeros(max(edges_cap, 1), np.int32)
        _check(lib().psb_slot_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(w),
                                          ctypes.byref(ob), ctypes.c_void_p(edges.ctypes.data), ctypes.c_int64(edges_cap),
                                          ctypes.byref(ne), ctypes.byref(st), ctypes.byref(lat)), "psb_slot_server_poll")
        if not done.value:
            return None
        return dict(weight=w.value, obs=ob.value, edges=edges[: min(ne.value, edges_cap)].copy(), n_edges=ne.value,
                    status=st.value, latency_ns=lat.value)

    def collect(self, max_n: int = 4096) -> list:
        t = np.zeros(max(max_n, 1), np.uint64); w = np.zeros_like(t, dtype=np.int64)
        ob = np.zeros_like(t); st = np.zeros(len(t), np.int32); lat = np.zeros(len(t), np.int64)
        P = lambda a: ctypes.c_void_p(a.ctypes.data)
        k = _check(lib().psb_slot_server_collect(self._h, ctypes.c_int32(max_n), P(t), P(w), P(ob), P(st), P(lat)),
                   "psb_slot_server_collect")
        return [dict(ticket=int(t[i]), weight=int(w[i]), obs=int(ob[i]), status=int(st[i]), latency_ns=int(lat[i]))
                for i in range(k)]

    def stats(self) -> dict:
        v = (ctypes.c_int64 * 5)()
        _check(lib().psb_slot_server_stats(self._h, v), "psb_slot_server_stats")
        return {"windows": v[0], "overflow_redecoded": v[1], "waiting": v[2], "in_flight": v[3], "slots": v[4]}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_slot_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StreamServer:
    """psb_stream_server: sliding-window decoding of live syndrome streams through the slot server.  Each of
    n_streams streams is one run of the layered graph `g`; push its layers as they arrive, poll for the
    committed result.  Close it before any device-wide synchronisation (its slot kernel keeps running)."""

    def __init__(self, g, layer_size: int, window_layers: int, commit_layers: int, n_streams: int, slots: int = 0,
                 **opts):
        u = np.ascontiguousarray(g.u, np.int32); v = np.ascontiguousarray(g.v, np.int32)
        w = np.ascontiguousarray(g.w, np.int32); o = np.ascontiguousarray(g.obs_mask, np.uint64)
        desc = _GraphDesc(g.num_detectors, len(u), u.ctypes.data, v.ctypes.data, w.ctypes.data, o.ctypes.data)
        c = _make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().psb_stream_server_create(ctypes.byref(desc), ctypes.c_int32(layer_size),
                                              ctypes.c_int32(window_layers), ctypes.c_int32(commit_layers),
                                              ctypes.byref(c), ctypes.c_int32(n_streams), ctypes.c_int32(slots),
                                              ctypes.byref(h)), "psb_stream_server_create")
        self._h = h
        nw, ns, nl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().psb_stream_server_info(h, ctypes.byref(nw), ctypes.byref(ns), ctypes.byref(nl)),
               "psb_stream_server_info")
        self.n_windows, self.n_shapes, self.n_layers = nw.value, ns.value, nl.value

    def push(self, stream: int, first_layer: int, n_layers: int, row):
        """row: the stream's packed syndrome row over the whole graph (only the pushed layers' bits are read)."""
        r = np.ascontiguousarray(row, np.uint8)
        _check(lib().psb_stream_push(self._h, ctypes.c_int32(stream), ctypes.c_int32(first_layer),
                                     ctypes.c_int32(n_layers), ctypes.c_void_p(r.ctypes.data)), "psb_stream_push")

    def push_many(self, streams, first_layer: int, n_layers: int, rows):
        """The same layer range of several streams in one call (rows[i] for streams[i])."""
        ids = np.ascontiguousarray(streams, np.int32)
        keep = [np.ascontiguousarray(r, np.uint8) for r in rows]
        ptrs = (ctypes.c_void_p * len(keep))(*[r.ctypes.data for r in keep])
        _check(lib().psb_stream_push_many(self._h, ctypes.c_int32(len(ids)), ctypes.c_void_p(ids.ctypes.data),
                                          ctypes.c_int32(first_layer), ctypes.c_int32(n_layers), ptrs),
               "psb_stream_push_many")

    def poll(self, stream: int) -> dict:
        done, cl, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        w, ob = ctypes.c_int64(), ctypes.c_uint64()
        _check(lib().psb_stream_poll(self._h, ctypes.c_int32(stream), ctypes.byref(done), ctypes.byref(cl),
                                     ctypes.byref(w), ctypes.byref(ob), ctypes.byref(st)), "psb_stream_poll")
        return dict(done=bool(done.value), committed_layers=cl.value, weight=w.value, obs=ob.value, status=st.value)

    def latencies(self, stream: int, decode: bool = False):
        """Nanoseconds from each committed window's last layer arriving to its commit; with decode=True also
        (second array) from its submission to the slot server to its decoded result."""
        n = ctypes.c_int32()
        buf = np.zeros(max(self.n_windows, 1), np.int64)
        dec = np.zeros_like(buf)
        _check(lib().psb_stream_latencies(self._h, ctypes.c_int32(stream), ctypes.c_int32(len(buf)),
                                          ctypes.c_void_p(buf.ctypes.data), ctypes.c_void_p(dec.ctypes.data),
                                          ctypes.byref(n)), "psb_stream_latencies")
        return (buf[: n.value].copy(), dec[: n.value].copy()) if decode else buf[: n.value].copy()

    def reset(self, stream: int):
        _check(lib().psb_stream_reset(self._h, ctypes.c_int32(stream)), "psb_stream_reset")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psb_stream_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
