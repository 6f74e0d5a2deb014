"""GPU: sliding windows fed by the serving loop (psb_stream_server), through
the C ABI.  Every stream's committed weight and observable equal the oracle's
windowed decode of the same syndrome, whatever order and chunking its layers
arrive in and whatever else is in flight.  No device-wide synchronisation
while a server exists (its slot kernel keeps running)."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import SEED, say

pytestmark = pytest.mark.gpu


def _run_streams(srv, rows, rng, limit_s=120, lockstep=False):
    """Pushes every stream's layers in random chunks, streams interleaved at random (or, lockstep, the same
    random chunk of every stream in one push_many call); waits for all."""
    n = len(rows)
    nxt = [0] * n
    while any(x < srv.n_layers for x in nxt):
        if lockstep:
            k = int(min(rng.integers(1, 5), srv.n_layers - nxt[0]))
            srv.push_many(list(range(n)), nxt[0], k, rows)
            nxt = [x + k for x in nxt]
            continue
        i = int(rng.integers(0, n))
        if nxt[i] >= srv.n_layers:
            continue
        k = int(min(rng.integers(1, 5), srv.n_layers - nxt[i]))
        srv.push(i, nxt[i], k, rows[i])
        nxt[i] += k
    t0 = time.time()
    res = [None] * n
    while time.time() - t0 < limit_s:
        res = [srv.poll(i) for i in range(n)]
        if all(r["done"] for r in res):
            break
        time.sleep(0.002)
    return res


@pytest.mark.parametrize("d,rounds,W,C,p,n", [(5, 20, 6, 3, 0.01, 60), (9, 27, 12, 6, 0.006, 40)])
def test_streams_equal_oracle_window_decode(d, rounds, W, C, p, n):
    """Two runs over the same streams (reset in between): layers pushed in
    random chunks of 1-4 with the streams interleaved at random, then in
    lockstep chunks through push_many.  Each stream ends done, with status OK
    and the oracle's committed weight and observable; every window has a
    latency record."""
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(d, p, rounds=rounds)
    L = (d * d - 1) // 2
    rows = synth.sample(g, n, seed=300 + d).syndromes
    sch = oracle.window_schedule(g, L, W, C)
    gs = [oracle.Graph(wg, SEED) for _, wg, _, _ in sch]
    want = [oracle.window_decode(g, sch, gs, L, synth.defects_of(rows[i], g.num_detectors)) for i in range(n)]
    srv = psb.StreamServer(g, L, W, C, n, tiebreak_seed=SEED)
    try:
        assert srv.n_windows == len(sch)
        for run in range(2):
            if run:
                for i in range(n):
                    srv.reset(i)
            res = _run_streams(srv, rows, np.random.default_rng(run), lockstep=run == 1)
            lats = [srv.latencies(i) for i in range(n)]
            say(f"d={d} run {run}: {sum(r['done'] for r in res)} of {n} streams done, "
                f"window latency p50 {np.median(np.concatenate(lats)) / 1e3:.1f} us")
            for i in range(n):
                w, o, ok = want[i]
                r = res[i]
                assert ok and r["done"] and r["status"] == 0, (run, i, r)
                assert (r["weight"], r["obs"], r["committed_layers"]) == (w, o, srv.n_layers), (run, i, r, w, o)
                assert len(lats[i]) == srv.n_windows and (lats[i] > 0).all()
    finally:
        srv.close()


def test_stream_push_refuses_out_of_order_layers():
    """Layers must arrive in order, each once; the refusal leaves the stream
    usable."""
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(5, 0.01, rounds=10)
    L = 12
    row = synth.sample(g, 1, seed=5).syndromes[0]
    srv = psb.StreamServer(g, L, 4, 2, 1, tiebreak_seed=SEED)
    try:
        with pytest.raises(psb.PsbError):
            srv.push(0, 1, 1, row)
        srv.push(0, 0, 2, row)
        with pytest.raises(psb.PsbError):
            srv.push(0, 0, 1, row)
        with pytest.raises(psb.PsbError):
            srv.push(0, 2, srv.n_layers, row)
        srv.push(0, 2, srv.n_layers - 2, row)
        t0 = time.time()
        while not srv.poll(0)["done"] and time.time() - t0 < 60:
            time.sleep(0.002)
        assert srv.poll(0)["done"] and srv.poll(0)["status"] == 0
    finally:
        srv.close()
