"""Benchmark: decoded shots/s and p50/p99 us per round on one MI355X.

Workload (default): rotated surface code d=21, 21 rounds, phenomenological
noise p=q=0.005, integer weights round(256 ln((1-p)/p)), 50,000 seeded shots
per step, all resident in HBM before timing.  A step = one persistent launch
that runs the whole hot path (syndrome intake, processing-cluster hierarchy,
hierarchical sparse-blossom execution, fuse and output) over the batch.

Prints one JSON line (see the field list in main()).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
DEVICE_CLOCK_HZ = 100e6        # wall_clock64() rate on gfx950


GRAPHS = {
    "phenom": "rotated surface code memory, phenomenological noise",
    "circuit_x": "rotated surface code Z memory, circuit-level X faults (CNOT order NW,SW,NE,SE)",
    "circuit_uniform": "rotated surface code X memory, uniform circuit-level noise (every circuit location p)",
    "circuit_physical": "rotated surface code X memory, physical circuit-level noise (1q gates p/10, idle noiseless)",
}


def make_graph(kind, d, p, q=None):
    """The detector graph of one of the workloads in GRAPHS (q: the phenomenological timelike rate, default p)."""
    import synth
    if kind == "phenom":
        return synth.rotated_phenom_graph(d, p, q=q)
    if kind == "circuit_x":
        return synth.rotated_circuit_x_graph(d, p)
    return synth.rotated_circuit_graph(d, p, kind.split("_", 1)[1])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_shot(nbytes, deg, n_explored, n_search, n_matched):
    """Algorithmic bytes of one shot (what the method has to move): the syndrome row, for every detector a region
    reaches its adjacency row (deg x (4 B neighbour + 4 B edge id + 4 B weight)) and its state written once (20 B),
    for every detector inside a level-1 exploring region its adjacency row (12 deg B), and the outputs (4 B per
    matched edge + 16 B)."""
    return nbytes + n_explored * (12 * deg + 20) + n_search * 12 * deg + 4 * n_matched + 16


def kernel_source_hash():
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2609_12262_amd", "csrc")
    # the decode kernels, their headers and the host code that lays out their state (not the serving runtime)
    files = sorted(glob.glob(os.path.join(csrc, "*.h"))
                   + [os.path.join(csrc, f) for f in ("psb_lib.hip", "psb_lane.hip")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def decoder_config_key(kw):
    """Decoder configuration with the library's defaults filled in (0 = default)."""
    tier = kw.get("first_tier", 0)
    nodes = kw.get("fast_max_nodes", 0) or 320
    regions = kw.get("fast_max_regions", 0) or (256 if tier else 208)
    lds = kw.get("fast_lds_state", 0) or 1           # 0 and 1 are the same placement
    q = kw.get("q", (1, 10))
    return f"first_tier={tier} state={nodes}/{regions} lds_state={lds} q={q[0]}/{q[1]}"


def measured_traffic(d, p, shots, kw):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this workload and
    decoder configuration, or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"psb_decode_kernel_d{d}_p{str(p).split('.')[1][:3]}_traffic.md")
    if (d, p, shots) != (21, 0.005, 50000) or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256",
                                                      "decoder_config"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash() or vals.get("decoder_config") != decoder_config_key(kw):
        return None
    return int(vals["traffic_bytes_per_launch"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_baseline(g, syndromes, rounds, seed, budget_s=20.0):
    """The oracle's serial sparse blossom on the host, in the same run and on the same shots as the GPU: global
    sparse blossom and partition-and-fuse, each on one core (per-shot latency) and on all cores of the box's
    share (one shot per task).  Bounded: each of the four legs stops after about a quarter of budget_s.  Also
    returns the oracle's per-shot counts (ARRIVE events, level-1 exploring-region detectors, matched edges) of
    the shots it decoded with partition-and-fuse."""
    import multiprocessing as mp
    import oracle
    import synth
    workers = max(1, min(16, os.cpu_count() or 1))
    og = oracle.Graph(g, seed)
    d_k, b_k, _ = oracle.schedule(max(og.tiebroken_weights()), levels=8)
    sb = oracle.SparseBlossom(g, seed)
    leg = budget_s / 4
    out = {"nproc": os.cpu_count(), "workers": workers, "cpu_model": cpu_model()}
    counts = []
    for name, glob in (("global", True), ("pf", False)):
        times = []
        t_end = time.perf_counter() + leg
        i = 0
        while time.perf_counter() < t_end and i < syndromes.shape[0]:
            dd = synth.defects_of(syndromes[i], g.num_detectors)
            t0 = time.perf_counter()
            r = sb.decode(dd, d_k, b_k, global_mode=glob)
            times.append(time.perf_counter() - t0)
            if not glob:
                counts.append((len(dd), r.arrivals, r.level1_search, len(r.edges), r.flags))
            i += 1
        us = np.asarray(times) * 1e6
        out[name + "_1core"] = {"shots": len(times), "shots_per_s": round(len(times) / float(np.sum(times)), 2),
                                "p50_us_per_round": round(float(np.percentile(us, 50)) / rounds, 2),
                                "p99_us_per_round": round(float(np.percentile(us, 99)) / rounds, 2)}
    ctx = mp.get_context("fork")
    for name, glob in (("global", True), ("pf", False)):
        chunk = 16
        t0 = time.time()
        done = 0
        with ctx.Pool(workers, initializer=_oracle_init, initargs=(g, seed, d_k, b_k, glob)) as pool:
            it = pool.imap_unordered(_oracle_chunk, [syndromes[s:s + chunk] for s in range(0, syndromes.shape[0], chunk)])
            for k in it:
                done += k
                if time.time() - t0 > leg:
                    pool.terminate()
                    break
        el = time.time() - t0
        out[name + "_all_cores"] = {"shots": done, "shots_per_s": round(done / el, 2)}
    return out, np.asarray(counts, np.int64)


_OG = None


def _oracle_init(g, seed, d_k, b_k, glob):
    global _OG
    import oracle
    _OG = (oracle.SparseBlossom(g, seed), g.num_detectors, d_k, b_k, glob)


def _oracle_chunk(rows):
    import synth
    sb, nd, d_k, b_k, glob = _OG
    for r in rows:
        sb.decode(synth.defects_of(r, nd), d_k, b_k, global_mode=glob)
    return len(rows)


def latency_scaling(args):
    """One shot per launch (the whole GPU holds one shot): per-round latency from launch to completion, per d."""
    import torch
    import synth
    import paper_2609_12262_amd as psb
    # the latency configuration's rate is 0.001 unless --latency-p (or a --p other than the headline's) is given
    p = args.latency_p if args.latency_p is not None else (args.p if args.p != 0.005 else 0.001)
    rows = []
    for d in [int(x) for x in args.latency.split(",")]:
        log(f"latency: building the {args.graph} graph, d={d}, p={p}")
        g = make_graph(args.graph, d, p)
        shots = synth.sample(g, args.latency_shots, seed=10 + d)
        G = psb.Graph.from_synth(g)
        synd = torch.from_numpy(shots.syndromes).cuda()
        kw = dict(tiebreak_seed=0x5EED, mode=args.mode, serial_level_one=1 if args.serial_level_one else 0,
                  cluster_walk=1 if args.cluster_walk else 0)
        if not args.no_autotune:
            # a batch of 64 shots, one per wavefront on an otherwise idle device, lasts about as long as its
            # slowest shot alone: the tuner's proxy for one-shot latency
            kw, _ = psb.autotune(G, synd[:64].contiguous(), reps=2, **kw)
        dec = psb.Decoder(G, **kw)
        out = dec.alloc(1, timestamps=True)
        stream = torch.cuda.current_stream()
        for i in range(min(3, args.latency_shots)):          # warm-up launches
            dec.decode_into(synd[i:i + 1], out)
        torch.cuda.synchronize()
        ev_ms, dev_us, ovf = [], [], 0
        for i in range(args.latency_shots):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            dec.decode_into(synd[i:i + 1], out)
            b.record(stream)
            b.synchronize()
            ev_ms.append(a.elapsed_time(b))
            td = out.t_done.cpu().numpy().astype(np.int64)
            dev_us.append((td[0] - td[1]) / DEVICE_CLOCK_HZ * 1e6)
            ovf += dec.last_overflow()
            if out.status.cpu().numpy()[0] != 0:
                log(f"WARNING: d={d} shot {i} status {out.status.cpu().numpy()[0]}")
        ev_us = np.array(ev_ms) * 1e3
        dev_us = np.array(dev_us)
        # parallel event count (E_ideal) of the same shots: one untimed batch with per-cluster accounting
        acc = psb.Decoder(G, **dict(kw, event_accounting=1))
        ao = acc.decode(synd, stats=True)
        torch.cuda.synchronize()
        ast = ao.stats.cpu().numpy()
        acc.close()
        rows.append({"d": d, "rounds": d, "detectors": g.num_detectors, "shots": args.latency_shots,
                     "decoder": {"first_tier_state": [kw.get("fast_max_nodes", 0), kw.get("fast_max_regions", 0)],
                                 "lds_state": kw.get("fast_lds_state", 0), "q": list(kw.get("q", (1, 10)))},
                     "defects_mean": float(np.unpackbits(shots.syndromes, axis=1, bitorder="little")
                                           [:, :g.num_detectors].sum(1).mean()),
                     "overflow_tier_shots": ovf,
                     "us_per_round_launch_p50": round(float(np.percentile(ev_us, 50)) / d, 3),
                     "us_per_round_launch_p99": round(float(np.percentile(ev_us, 99)) / d, 3),
                     "us_per_round_device_p50": round(float(np.percentile(dev_us, 50)) / d, 3),
                     "us_per_round_device_p99": round(float(np.percentile(dev_us, 99)) / d, 3),
                     "events_per_round_mean": round(float(ast[:, 8].mean()) / d, 3),
                     "e_ideal_per_round_mean": round(float(ast[:, 9].mean()) / d, 3),
                     "e_ideal_per_round_p99": round(float(np.percentile(ast[:, 9], 99)) / d, 3),
                     "clusters_mean": round(float(ast[:, 10].mean()), 2)})
        log(f"d={d}: {rows[-1]}")
        dec.close(); G.close()
    print(json.dumps({"metric": "one-shot-per-launch latency, us per round", "graph": GRAPHS[args.graph], "p": p,
                      "mode": args.mode,
                      "basis": "launch = HIP events around the launch on its stream; device = kernel start stamp "
                               "to shot completion (device clock)", "per_d": rows}), flush=True)


def serving(args):
    """Windows arrive one at a time (Poisson) at a mixed set of distances and noise rates; the server batches
    them per graph.  Latency per window = submit to completion (server clock), reported per round.  The same
    stream is then decoded in the one-shot-per-launch form (one window per launch, in arrival order)."""
    import ctypes
    import torch
    import synth
    import paper_2609_12262_amd as psb
    rng = np.random.default_rng(6)
    ds = [int(x) for x in args.serve_dists.split(",")]
    p_lo, p_hi = (float(x) for x in args.serve_p.split(","))
    gs = [synth.rotated_phenom_graph(d, 0.004) for d in ds]
    n = args.serve
    kind = rng.integers(0, len(ds), n)
    ps = rng.uniform(p_lo, p_hi, n)
    log(f"sampling {n} windows")
    rows, ws = [], []
    for i in range(n):
        g = gs[kind[i]]
        gp = synth.DetectorGraph(g.num_detectors, g.u, g.v, g.w, g.obs_mask, np.full(g.num_edges, ps[i]))
        rows.append(synth.sample(gp, 1, seed=5000 + i).syndromes[0])
        ws.append(synth.weight_from_p(float(ps[i])))
    Gs = [psb.Graph.from_synth(g) for g in gs]
    # windows carry a uniform weight, so they decode on unit-weight graphs: tune and compare there
    units = [psb.Graph.from_synth(synth.DetectorGraph(g.num_detectors, g.u, g.v, np.ones(g.num_edges, np.int32),
                                                       g.obs_mask, g.p)) for g in gs]
    base = dict(tiebreak_seed=0x5EED, num_slots=1024, overflow_slots=256, edges_per_shot=1024)
    opts, tuned = [], {}
    for j, d in enumerate(ds):
        if args.no_autotune:
            opts.append(base)
            continue
        sel = [r for r, k in zip(rows, kind) if k == j][:2048]
        best, _ = psb.autotune(units[j], torch.from_numpy(np.stack(sel)).cuda(), reps=1, **base)
        opts.append(best)
        tuned[str(d)] = {"first_tier": best["first_tier"], "state": [best["fast_max_nodes"], best["fast_max_regions"]],
                         "lds_state": best["fast_lds_state"], "q": list(best["q"])}
    log(f"autotuned {tuned}")
    srv = psb.Server(Gs, opts=opts)
    psb.lib()
    rep = ctypes.CDLL(os.path.join(ROOT, "paper_2609_12262_amd", "libpsb_replay.so"))
    rep.psb_replay.restype = ctypes.c_int32
    rep.psb_replay_oneshot.restype = ctypes.c_int32
    rows = [np.ascontiguousarray(r) for r in rows]
    syn_ptrs = (ctypes.c_void_p * n)(*[r.ctypes.data for r in rows])
    wts = np.ascontiguousarray(ws, np.int32)
    gidx = np.ascontiguousarray(kind, np.int32)

    def run(arrivals):
        lat = np.zeros(n, np.int64)
        st = np.zeros(n, np.int32)
        span, wall = ctypes.c_double(), ctypes.c_double()
        arr = None if arrivals is None else np.ascontiguousarray(arrivals, np.float64)
        rc = rep.psb_replay(srv._h, ctypes.c_int64(n), ctypes.c_void_p(gidx.ctypes.data), syn_ptrs,
                            ctypes.c_void_p(wts.ctypes.data),
                            ctypes.c_void_p(arr.ctypes.data) if arr is not None else ctypes.c_void_p(0),
                            ctypes.c_void_p(lat.ctypes.data), ctypes.c_void_p(st.ctypes.data),
                            ctypes.byref(span), ctypes.byref(wall))
        if rc != 0:
            raise RuntimeError(f"psb_replay failed ({rc})")
        if not (st == 0).all():
            log(f"WARNING: statuses {np.bincount(st)}")
        return lat, span.value, wall.value

    run(None)                                             # warm-up: builds the unit-weight decoders
    s0 = srv.stats()
    lat, _, wall = run(None)
    s1 = srv.stats()
    capacity = n / wall
    rate = args.serve_load * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    log(f"capacity {capacity:.0f} windows/s; offering {rate:.0f} windows/s")
    lat, t_sub, wall = run(arrivals)
    s2 = srv.stats()
    offered = n / t_sub
    # the same stream at each load of the sweep (offered rate = load x the batched capacity above)
    sweep = {}
    loads = [float(x) for x in args.serve_loads.split(",")] if args.serve_loads else []
    for ld in loads:
        arr_l = np.cumsum(np.random.default_rng(7).exponential(1.0 / (ld * capacity), n))
        lat_l, t_sub_l, _ = run(arr_l)
        sweep[str(ld)] = {"offered_windows_per_s": round(n / t_sub_l, 1),
                          "p50_us_per_round": round(float(np.percentile(lat_l / 1e3 / np.asarray(ds)[kind], 50)), 3),
                          "p99_us_per_round": round(float(np.percentile(lat_l / 1e3 / np.asarray(ds)[kind], 99)), 3)}
        log(f"pipe server, load {ld}: {sweep[str(ld)]}")
    srv.close()

    # slot-level server: one persistent kernel, windows taken one at a time as slots free up
    slot_out = None
    if not args.no_slot_server:
        ssrv = psb.SlotServer(Gs, opts=opts, waves=args.slot_waves)
        rep.psb_replay_slots.restype = ctypes.c_int32

        def run_slots(arrivals_s):
            lat_s = np.zeros(n, np.int64)
            st_s = np.zeros(n, np.int32)
            span, wall_s_ = ctypes.c_double(), ctypes.c_double()
            arr = None if arrivals_s is None else np.ascontiguousarray(arrivals_s, np.float64)
            rc = rep.psb_replay_slots(ssrv._h, ctypes.c_int64(n), ctypes.c_void_p(gidx.ctypes.data), syn_ptrs,
                                      ctypes.c_void_p(wts.ctypes.data),
                                      ctypes.c_void_p(arr.ctypes.data) if arr is not None else ctypes.c_void_p(0),
                                      ctypes.c_void_p(lat_s.ctypes.data), ctypes.c_void_p(st_s.ctypes.data),
                                      ctypes.byref(span), ctypes.byref(wall_s_))
            if rc != 0:
                raise RuntimeError(f"psb_replay_slots failed ({rc})")
            if not (st_s == 0).all():
                log(f"WARNING: slot server statuses {np.bincount(st_s)}")
            return lat_s, span.value, wall_s_.value

        run_slots(None)                                   # warm-up
        _, _, wall_cap = run_slots(None)
        slot_out = {"capacity_windows_per_s": round(n / wall_cap, 1), "slots": ssrv.stats()["slots"], "loads": {}}
        for ld in sorted(set(loads + [args.serve_load])):
            arr_l = np.cumsum(np.random.default_rng(7).exponential(1.0 / (ld * capacity), n))
            lat_l, t_sub_l, _ = run_slots(arr_l)
            pr = lat_l / 1e3 / np.asarray(ds)[kind]
            slot_out["loads"][str(ld)] = {
                "offered_windows_per_s": round(n / t_sub_l, 1),
                "p50_us_per_round": round(float(np.percentile(pr, 50)), 3),
                "p99_us_per_round": round(float(np.percentile(pr, 99)), 3),
                "per_d": {str(d): {"p50_us_per_round": round(float(np.percentile(pr[kind == j], 50)), 3),
                                   "p99_us_per_round": round(float(np.percentile(pr[kind == j], 99)), 3)}
                          for j, d in enumerate(ds)}}
            log(f"slot server, load {ld}: p50 {slot_out['loads'][str(ld)]['p50_us_per_round']} "
                f"p99 {slot_out['loads'][str(ld)]['p99_us_per_round']} us/round")
        slot_out["stats"] = ssrv.stats()
        ssrv.close()

    def delta(a, b):
        nb, nw = b["batches"] - a["batches"], b["windows"] - a["windows"]
        return {"batches": nb, "mean_batch": round(nw / max(nb, 1), 1),
                "mean_queue_us": round((b["mean_queue_us"] * b["windows"] - a["mean_queue_us"] * a["windows"]) / max(nw, 1), 1),
                "mean_batch_run_us": round((b["mean_batch_run_us"] * b["batches"] - a["mean_batch_run_us"] * a["batches"]) / max(nb, 1), 1),
                "mean_launch_us": round((b["mean_launch_us"] * b["batches"] - a["mean_launch_us"] * a["batches"]) / max(nb, 1), 1)}

    dv = np.asarray(ds)[kind]
    per_round = lat / 1e3 / dv

    def pct(x, q):
        return round(float(np.percentile(x, q)), 3)

    # one-shot-per-launch form: the first m windows of the same stream
    m = min(n, args.oneshot_windows)
    decs = [psb.Decoder(u, tiebreak_seed=0x5EED) for u in units]
    dec_arr = (ctypes.c_void_p * len(decs))(*[dd._h.value for dd in decs])
    nbytes = np.ascontiguousarray([u.syndrome_bytes for u in units], np.int32)

    def run1(arr):
        lat1 = np.zeros(m, np.int64)
        st1 = np.zeros(m, np.int32)
        wall1 = ctypes.c_double()
        a1 = None if arr is None else np.ascontiguousarray(arr[:m], np.float64)
        rc = rep.psb_replay_oneshot(dec_arr, ctypes.c_int32(len(decs)), ctypes.c_int64(m),
                                    ctypes.c_void_p(gidx.ctypes.data), syn_ptrs, ctypes.c_void_p(nbytes.ctypes.data),
                                    ctypes.c_void_p(a1.ctypes.data) if a1 is not None else ctypes.c_void_p(0),
                                    ctypes.c_void_p(lat1.ctypes.data), ctypes.c_void_p(st1.ctypes.data),
                                    ctypes.byref(wall1))
        if rc != 0:
            raise RuntimeError(f"psb_replay_oneshot failed ({rc})")
        return lat1, wall1.value

    log(f"one-shot-per-launch form on {m} windows")
    run1(None)
    lat1, wall1 = run1(None)
    cap1 = m / wall1
    lat1q, _ = run1(arrivals)
    pr1 = lat1q / 1e3 / dv[:m]
    pr1_alone = lat1 / 1e3 / dv[:m]
    for dd in decs:
        dd.close()
    out = {"metric": "serving: window latency, us per round (submit to completion)", "windows": n,
           "distances": ds, "p_range": [p_lo, p_hi], "capacity_windows_per_s": round(capacity, 1),
           "target_load": args.serve_load, "offered_windows_per_s": round(offered, 1),
           "p50_us_per_round": pct(per_round, 50), "p99_us_per_round": pct(per_round, 99),
           "per_d": {str(d): {"p50_us_per_round": pct(per_round[kind == j], 50),
                              "p99_us_per_round": pct(per_round[kind == j], 99)}
                     for j, d in enumerate(ds)},
           "autotuned": tuned,
           "server_capacity_run": delta(s0, s1), "server_load_run": delta(s1, s2),
           "load_sweep": sweep, "slot_server": slot_out,
           "one_shot_per_launch": {
               "windows": m, "capacity_windows_per_s": round(cap1, 1),
               "alone_p50_us_per_round": pct(pr1_alone, 50), "alone_p99_us_per_round": pct(pr1_alone, 99),
               "same_stream_p50_us_per_round": pct(pr1, 50), "same_stream_p99_us_per_round": pct(pr1, 99),
               "basis": "one window per psb_decode_batch launch in arrival order (copy in, decode, copy out, "
                        "wait); 'alone' = back to back without queueing, 'same_stream' = the first windows of "
                        "the served Poisson stream, queueing included"},
           "driver": "native replay thread (libpsb_replay.so): submits at the arrival times, a second thread "
                     "collects completions"}
    print(json.dumps(out), flush=True)


def sliding_window(args):
    """Sliding-window decoding of long streams: B shots of R rounds each, windows of W layers committing C.
    Sustained throughput = rounds decoded per second over the whole batch."""
    import torch
    import synth
    import paper_2609_12262_amd as psb
    d, R, W, C = (int(x) for x in args.window.split(","))
    g = synth.rotated_phenom_graph(d, args.p, rounds=R)
    L = (d * d - 1) // 2
    log(f"sampling {args.shots} shots d={d} rounds={R} p={args.p}")
    shots = synth.sample(g, args.shots, seed=7)
    caps = [int(x) for x in args.window_caps.split(",")] if args.window_caps else [0, 0]
    plan = psb.WindowPlan(g, L, W, C, tiebreak_seed=0x5EED, fast_max_nodes=caps[0], fast_max_regions=caps[1])
    synd = torch.from_numpy(shots.syndromes).cuda()
    for _ in range(args.warmup):
        out = plan.decode(synd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = plan.decode(synd)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    st = out["status"].cpu().numpy()
    print(json.dumps({"metric": "sliding-window decoding: rounds per second", "d": d, "rounds": R,
                      "window_layers": W, "commit_layers": C, "p": args.p, "shots": args.shots,
                      "windows": plan.n_windows, "window_graphs": plan.n_shapes, "first_tier_state": caps,
                      "value": round(args.shots * R / wall, 1), "unit": "rounds/s",
                      "ms_per_batch": round(wall * 1e3, 3), "us_per_window_launch": round(wall * 1e6 / plan.n_windows, 1),
                      "ok_shots": int((st == 0).sum())}), flush=True)
    plan.close()


def streaming(args):
    """Sliding windows fed by the serving loop: --streams streams of R rounds each, every stream's rounds pushed
    at the syndrome rate (one round per --round-us microseconds) and decoded window by window through the slot
    server as they complete.  Per rate: offered and sustained rounds/s over all streams, the lag of the last
    commit behind the last round, each window's latency from its last round's arrival to its commit, and its
    decode time (submission to the slot server to its decoded result)."""
    import ctypes
    import synth
    import paper_2609_12262_amd as psb
    d, R, W, C = (int(x) for x in args.stream.split(","))
    g = synth.rotated_phenom_graph(d, args.p, rounds=R)
    L = (d * d - 1) // 2
    n = args.streams
    log(f"sampling {n} streams d={d} rounds={R} p={args.p}")
    rows = synth.sample(g, n, seed=9).syndromes
    caps = [int(x) for x in args.window_caps.split(",")] if args.window_caps else [0, 0]
    srv = psb.StreamServer(g, L, W, C, n, tiebreak_seed=0x5EED, fast_max_nodes=caps[0], fast_max_regions=caps[1],
                           fast_lds_state=args.lds_state)
    rep = ctypes.CDLL(os.path.join(ROOT, "paper_2609_12262_amd", "libpsb_replay.so"))
    rep.psb_stream_replay.restype = ctypes.c_int32
    keep = [np.ascontiguousarray(r) for r in rows]
    ptrs = (ctypes.c_void_p * n)(*[r.ctypes.data for r in keep])
    out = {"metric": "streaming sliding-window decoding: sustained rounds/s against the syndrome rate",
           "d": d, "rounds": R, "window_layers": W, "commit_layers": C, "p": args.p, "streams": n,
           "windows_per_stream": srv.n_windows, "first_tier_state": caps, "lds_state": args.lds_state, "rates": {}}
    for ru in [float(x) for x in args.round_us.split(",")] + [float(args.round_us.split(",")[0])]:
        for i in range(n):
            srv.reset(i)
        wall, span = ctypes.c_double(), ctypes.c_double()
        rc = rep.psb_stream_replay(srv._h, ctypes.c_int32(n), ptrs, ctypes.c_int32(srv.n_layers),
                                   ctypes.c_int32(args.layers_per_push), ctypes.c_double(ru * 1e-6),
                                   ctypes.c_double(120.0), ctypes.byref(wall), ctypes.byref(span))
        if rc != 0:
            raise RuntimeError(f"psb_stream_replay failed ({rc})")
        res = [srv.poll(i) for i in range(n)]
        ld = [srv.latencies(i, decode=True) for i in range(n)]
        lat = np.concatenate([x[0] for x in ld]) / 1e3
        dec = np.concatenate([x[1] for x in ld]) / 1e3
        ok = sum(1 for r in res if r["done"] and r["status"] == 0)
        rec = {"round_us": ru, "offered_rounds_per_s": round(n * 1e6 / ru, 1) if ru > 0 else None,
               "pushed_rounds_per_s": round(n * srv.n_layers / span.value, 1),
               "sustained_rounds_per_s": round(n * srv.n_layers / wall.value, 1),
               "lag_after_last_round_us": round((wall.value - span.value) * 1e6, 1),
               "window_latency_us_p50": round(float(np.percentile(lat, 50)), 1),
               "window_latency_us_p99": round(float(np.percentile(lat, 99)), 1),
               "window_decode_us_p50": round(float(np.percentile(dec, 50)), 1),
               "window_decode_us_p99": round(float(np.percentile(dec, 99)), 1), "ok_streams": ok}
        log(f"round every {ru} us: {rec}")
        out["rates"][str(ru)] = rec          # the first rate runs twice; the second run (warm) is kept
    srv.close()
    print(json.dumps(out), flush=True)


def complementary(args):
    """Complementary-gap decoding of a batch: two constrained MWEM decodes per shot (observable 0 and 1)."""
    import torch
    import synth
    import paper_2609_12262_amd as psb
    g = make_graph(args.graph, args.d, args.p, args.q)
    log(f"sampling {args.shots} shots d={args.d} p={args.p} graph={args.graph}")
    shots = synth.sample(g, args.shots, seed=3)
    plan = psb.ComplementaryPlan(g, 0, tiebreak_seed=0x5EED)
    synd = torch.from_numpy(shots.syndromes).cuda()
    for _ in range(args.warmup):
        out = plan.decode(synd)
        torch.cuda.synchronize()
        log("warm-up batch done")
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = plan.decode(synd)
        torch.cuda.synchronize()
        log(f"batch {k} done")
    wall = (time.perf_counter() - t0) / args.steps
    gap = out["gap"].cpu().numpy()
    st = out["status"].cpu().numpy()
    print(json.dumps({"metric": "complementary-gap decoding: shots per second (two constrained decodes each)",
                      "graph": args.graph, "d": args.d, "p": args.p, "shots": args.shots,
                      "value": round(args.shots / wall, 1), "unit": "shots/s", "ms_per_batch": round(wall * 1e3, 3),
                      "gap_p50": float(np.percentile(gap, 50)), "gap_p01": float(np.percentile(gap, 1)),
                      "ok_shots": int((st == 0).sum())}), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--d", type=int, default=21)
    ap.add_argument("--p", type=float, default=0.005)
    ap.add_argument("--q", type=float, default=None, help="phenomenological graphs: timelike rate (default p)")
    ap.add_argument("--shots", type=int, default=50000)
    ap.add_argument("--mode", type=int, default=0, help="0 partition-and-fuse, 1 global sparse blossom")
    ap.add_argument("--graph", default="phenom", choices=list(GRAPHS),
                    help="phenomenological graph; circuit-level X-fault graph of Z memory (diagonal edges, mixed "
                         "weights); or X-memory graph under the uniform or physical circuit-level noise model")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--serial-level-one", action="store_true",
                    help="send every level-1 processing cluster through the event loop (no concurrent level-1 pass)")
    ap.add_argument("--cluster-walk", action="store_true",
                    help="the clustering search walks its paths at every level (no ball tables)")
    ap.add_argument("--no-autotune", action="store_true", help="default decoder configuration instead of the "
                                                                 "autotuner's pick")
    ap.add_argument("--no-graph", action="store_true", help="eager psb_decode_batch launches instead of a "
                                                              "captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (3 times): the reference "
                         "kernel that scales rocprof FETCH_SIZE / WRITE_SIZE readings to bytes")
    ap.add_argument("--latency", type=str, default="",
                    help="latency-scaling mode: comma-separated distances (e.g. 11,21,31,41,51); every shot is "
                         "decoded alone, one launch per shot, at p=q=--p (default 0.001 in this mode)")
    ap.add_argument("--latency-shots", type=int, default=200)
    ap.add_argument("--latency-p", type=float, default=None,
                    help="noise rate of --latency (default 0.001, or --p when it is not the headline's 0.005)")
    ap.add_argument("--serve", type=int, default=0,
                    help="serving mode: this many windows with d in {9,13,17,21,25} (d rounds) and p ~ U[0.001, "
                         "0.007] (uniform per-window weight), Poisson arrivals at --serve-load x the measured "
                         "capacity for the mix")
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-loads", default="0.3,0.7,0.9",
                    help="further offered loads (x the batched capacity) run with both serving runtimes")
    ap.add_argument("--no-slot-server", action="store_true", help="skip the slot-level server in --serve")
    ap.add_argument("--slot-waves", type=int, default=0, help="slots of the slot-level server (0 = as many as fit)")
    ap.add_argument("--serve-dists", default="9,13,17,21,25")
    ap.add_argument("--serve-p", default="0.001,0.007", help="window noise rates drawn uniformly from this range")
    ap.add_argument("--oneshot-windows", type=int, default=3000)
    ap.add_argument("--window", default="", help="d,rounds,W,C: sliding-window decoding of --shots long streams")
    ap.add_argument("--stream", default="", help="d,rounds,W,C: sliding windows fed by the serving loop")
    ap.add_argument("--streams", type=int, default=64, help="streams for --stream")
    ap.add_argument("--round-us", default="0", help="--stream: microseconds per syndrome round (list; 0 = as fast "
                                                   "as the pushes go)")
    ap.add_argument("--layers-per-push", type=int, default=1)
    ap.add_argument("--lds-state", type=int, default=3, help="--stream: first-tier state placement of the window "
                                                             "decoders (fast_lds_state; 3 = all per-shot state in LDS)")
    ap.add_argument("--complementary", action="store_true",
                    help="complementary-gap decoding (both values of the logical observable) of --shots shots")
    ap.add_argument("--window-caps", default="640,416",
                    help="nodes,regions of the window decoders' first tier (the best of a sweep at d=21, W=2d)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for {args.gpus}): shots and windows shard across GPUs with no "
              "exchange, but only the one-GPU share is implemented and measured.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serving(args)
        return
    if args.window:
        sliding_window(args)
        return
    if args.stream:
        streaming(args)
        return
    if args.complementary:
        complementary(args)
        return
    if args.latency:
        latency_scaling(args)
        return
    if args.copy_calibration_mib > 0:
        import torch
        n = args.copy_calibration_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n}), flush=True)
        return

    import torch
    import synth
    import paper_2609_12262_amd as psb

    seed_sample = {0.005: 3, 0.001: 4}.get(args.p, 3)
    g = make_graph(args.graph, args.d, args.p, args.q)
    log(f"sampling {args.shots} shots d={args.d} p={args.p} graph={args.graph}")
    shots = synth.sample(g, args.shots, seed=seed_sample)
    G = psb.Graph.from_synth(g)
    synd = torch.from_numpy(shots.syndromes).cuda()
    base = dict(tiebreak_seed=0x5EED, mode=args.mode, num_slots=args.slots,
                serial_level_one=1 if args.serial_level_one else 0, cluster_walk=1 if args.cluster_walk else 0)
    tune_table = None
    if args.no_autotune:
        kw = base
    else:
        log("autotune")
        kw, tune_table = psb.autotune(G, synd, reps=1, **base)
    dec = psb.Decoder(G, **kw)
    out = dec.alloc(args.shots, timestamps=True, stats=True)
    stream = torch.cuda.current_stream()
    if args.no_graph:
        step = lambda: dec.decode_into(synd, out, stream)
    else:
        bg = dec.capture(synd, out)
        step = lambda: bg.launch(stream)
    torch.cuda.synchronize()
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    status = out.status.cpu().numpy()
    if not (status == 0).all():
        log(f"WARNING: non-zero statuses {np.bincount(status)}")
    stats = out.stats.cpu().numpy()
    ne = out.n_edges.cpu().numpy()
    td = out.t_done.cpu().numpy().astype(np.int64)
    lat_us = (td[:-1] - td[-1]) / DEVICE_CLOCK_HZ * 1e6
    per_round = lat_us / args.d
    ms_per_step = wall * 1e3 / args.steps
    # every step decodes the same batch: shots that end with a non-zero status (capacity, truncation) are not
    # counted as decoded
    n_ok = int((status == 0).sum())
    value = n_ok * args.steps / wall
    deg = int(np.bincount(np.concatenate([g.u, g.v[g.v >= 0]]), minlength=g.num_detectors).max())
    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    # kernel-counted work: detectors reached (events + arrivals) and clustering-search adjacency entries
    kern_bytes = int(sum(bytes_per_shot(g.nbytes, deg, int(stats[i, 1]), 0, int(ne[i])) for i in range(len(stats)))
                     + 12 * int(stats[:, 2].astype(np.int64).sum()))
    line = {
        "metric": "decoded shots/sec and p50/p99 us per round at d=21, d rounds, p=0.5%",
        "value": round(value, 1),
        "unit": "shots/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "decoded_shots_per_step": n_ok,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int128", "data": "synthetic",
        "config": {"workload": (f"{GRAPHS[args.graph]}, d={args.d}, {args.d} rounds, "
                                f"{('p=q' if args.q is None else 'p') if args.graph == 'phenom' else 'p'}={args.p}"
                                f"{'' if args.q is None else f', q={args.q}'}, {args.shots} shots per step, "
                                f"one persistent launch"),
                   "d": args.d, "rounds": args.d, "p": args.p, "shots_per_step": args.shots,
                   "mode": "partition-and-fuse" if args.mode == 0 else "global sparse blossom",
                   "level_one": ("event loop" if args.serial_level_one else
                                 "single-event clusters in one concurrent pass, the rest in the event loop"),
                   "cluster_search": ("walks its paths" if args.cluster_walk else
                                      "ball tables for levels of at most two edges, else walks"),
                   "first_tier": "one shot per lane" if kw.get("first_tier", 0) else "one shot per wavefront",
                   "first_tier_state": [kw.get("fast_max_nodes", 0), kw.get("fast_max_regions", 0)],
                   "first_tier_lds_state": kw.get("fast_lds_state", 0),
                   "schedule_q": list(kw.get("q", (1, 10))),
                   "first_tier_slots": dec.fast_slots, "overflow_tier_slots": dec.overflow_slots,
                   "overflow_shots": dec.last_overflow(), "hip_graph": not args.no_graph,
                   "autotune": None if tune_table is None else
                   [{"first_tier": t["first_tier"], "state": [t["fast_max_nodes"], t["fast_max_regions"]],
                     "lds_state": t["fast_lds_state"], "q": list(t["q"]), "ms": t["ms"], "status": t["status"]}
                    for t in tune_table]},
        "latency_us_per_round": {"p50": round(float(np.percentile(per_round, 50)), 3),
                                 "p99": round(float(np.percentile(per_round, 99)), 3),
                                 "basis": "batch submission to shot completion (device clock), last step"},
        "work_per_shot": {"events": float(stats[:, 0].mean()), "reached": float(stats[:, 1].mean()),
                          "cluster_visits": float(stats[:, 2].mean()), "log_records": float(stats[:, 3].mean()),
                          "us_intake_cluster": float(stats[:, 4].mean()) * 1e6 / DEVICE_CLOCK_HZ,
                          "us_dynamics": float(stats[:, 5].mean()) * 1e6 / DEVICE_CLOCK_HZ,
                          "us_fuse": float(stats[:, 6].mean()) * 1e6 / DEVICE_CLOCK_HZ,
                          "us_shot": float(stats[:, 7].mean()) * 1e6 / DEVICE_CLOCK_HZ},
    }
    roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
            "traffic": measured_traffic(args.d, args.p, args.shots, kw) if args.graph == "phenom" else None,
            "avg_launch_ms": round(avg_launch_s * 1e3, 3),
            "kernel": "psb_lane_kernel" if kw.get("first_tier", 0) else "psb_decode_kernel<0, 0, 0>",
            "alg_bytes_per_launch_kernel_counts": kern_bytes,
            "achieved_kernel_counts": round(kern_bytes / avg_launch_s / 1e9, 2)}
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        log("cpu baseline (oracle: serial sparse blossom, global and partition-and-fuse)")
        cb, counts = cpu_oracle_baseline(g, shots.syndromes, args.d, 0x5EED, args.cpu_budget)
        ok = counts[counts[:, 4] == 0]
        n_def, n_arr, n_srch, n_m = (float(ok[:, k].mean()) for k in range(4))
        per_shot = bytes_per_shot(g.nbytes, deg, n_def + n_arr, n_srch, n_m)
        alg = per_shot * args.shots
        roof.update({"achieved": round(alg / avg_launch_s / 1e9, 2), "frac": round(alg / avg_launch_s / 1e9 / HBM_PEAK_GBS, 5),
                     "alg_bytes_per_launch": int(alg),
                     "alg_bytes_basis": {"shots_sampled": int(len(ok)), "detection_events": round(n_def, 2),
                                         "arrivals": round(n_arr, 2), "level1_search_detectors": round(n_srch, 2),
                                         "matched_edges": round(n_m, 2), "deg": deg, "syndrome_bytes": g.nbytes,
                                         "bytes_per_shot": round(per_shot, 1),
                                         "source": "oracle partition-and-fuse counts on the cpu_baseline sample"}})
        line["cpu_baseline"] = {"value": cb["global_all_cores"]["shots_per_s"], "unit": "shots/s",
                                "cores": cb["workers"], "kind": "oracle",
                                "sample": (f"first shots of the same batch, serial global sparse blossom (C), about "
                                           f"{args.cpu_budget / 4:.0f} s per leg: {cb['global_all_cores']['shots']} "
                                           f"shots on {cb['workers']} processes"),
                                **{k: v for k, v in cb.items() if k not in ("workers",)}}
    else:
        roof.update({"achieved": roof["achieved_kernel_counts"],
                     "frac": round(roof["achieved_kernel_counts"] / HBM_PEAK_GBS, 5),
                     "alg_bytes_per_launch": kern_bytes,
                     "alg_bytes_basis": {"source": "kernel counters (no cpu_baseline leg in this run)"}})
    line["roofline"] = roof
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
