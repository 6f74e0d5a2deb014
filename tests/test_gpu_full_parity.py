"""GPU parity over every shot of the benchmark's launch shape, and at the
latency configuration's largest distances.

Every shot is compared with the serial sparse-blossom oracle (fast enough to
decode 50,000 d=21 shots in seconds on the host cores; it is itself pinned to
the Dijkstra + Edmonds MWEM), and a sample with the Dijkstra + Edmonds oracle
directly."""
import numpy as np
import pytest

import synth
from gpu_helpers import SEED, compare, compare_parallel, compare_sb_parallel, gpu_decode, say

pytestmark = pytest.mark.gpu


def _every_shot(g, syndromes, res, label):
    n = syndromes.shape[0]
    bad = compare_sb_parallel(g, syndromes, res, range(n))
    say(f"{label}: {n} shots against the sparse-blossom oracle, {len(bad)} differ")
    assert not bad, bad[:5]
    rng = np.random.default_rng(1)
    idx = sorted(rng.choice(n, 400, replace=False).tolist())
    bad = compare_parallel(g, syndromes, res, idx, workers=16, chunk=25)
    say(f"{label}: {len(idx)} sampled shots against the Dijkstra + Edmonds oracle, {len(bad)} differ")
    assert not bad, bad[:5]


@pytest.mark.parametrize("p,seed", [(0.005, 3), (0.001, 4)])
def test_d21_every_shot_of_the_benchmark_launch(p, seed):
    """d=21, 21 rounds, 50,000 shots in one launch with the library's default
    decoder (the configuration the autotuner picks for the benchmark): the
    edge set, weight and observable of every shot equal the oracle's."""
    g = synth.rotated_phenom_graph(21, p)
    s = synth.sample(g, 50000, seed=seed)
    say(f"d21 p={p}: decoding 50000 shots")
    res = gpu_decode(g, s.syndromes)
    _every_shot(g, s.syndromes, res, f"d21 p={p}")


def test_d21_circuit_uniform_every_shot():
    """The paper's workload shape: X-memory graph under uniform circuit-level
    noise, d=21, 21 rounds, p=0.001, 50,000 shots in one launch with the
    default decoder: every shot equals the oracle."""
    g = synth.rotated_circuit_graph(21, 0.001, "uniform")
    s = synth.sample(g, 50000, seed=160)
    say("d21 circuit uniform p=0.001: decoding 50000 shots")
    res = gpu_decode(g, s.syndromes)
    _every_shot(g, s.syndromes, res, "d21 circuit uniform")


@pytest.mark.parametrize("d", [31, 51])
def test_latency_configuration_one_launch_per_shot(d):
    """The latency measurement's configuration at d=31 and d=51 (p=q=0.001,
    the seeds bench.py uses): the decoder the autotuner picks on a 64-shot
    sample, one launch per shot as timed, 64 shots, every one equal to the
    Dijkstra + Edmonds oracle."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(d, 0.001)
    s = synth.sample(g, 64, seed=10 + d)
    G = psb.Graph.from_synth(g)
    synd = torch.from_numpy(s.syndromes).cuda()
    kw, _ = psb.autotune(G, synd, reps=1, tiebreak_seed=SEED)
    say(f"d={d}: autotuned {kw}")
    dec = psb.Decoder(G, **kw)
    out = dec.alloc(1)
    rows = []
    for i in range(64):
        dec.decode_into(synd[i:i + 1], out)
        torch.cuda.synchronize()
        rows.append({k: getattr(out, k).cpu().numpy()[0].copy() for k in ("edges", "n_edges", "weight", "obs", "status")})
    dec.close(); G.close()
    res = {k: np.stack([r[k] for r in rows]) for k in rows[0]}
    res["obs"] = res["obs"].view(np.uint64)
    bad = compare_parallel(g, s.syndromes, res, range(64), workers=16, chunk=4)
    assert not bad, bad[:5]


def test_d5_config_one_launch_per_shot():
    """d=5, 5 rounds, p=q=0.005, 10,000 shots decoded one launch per shot (the
    one-shot-per-launch form of the small configuration): every shot equals
    the oracle."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(5, 0.005)
    s = synth.sample(g, 10000, seed=1)
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=SEED)
    synd = torch.from_numpy(s.syndromes).cuda()
    n = 10000
    res = {"edges": np.zeros((n, dec.edges_per_shot), np.int32), "n_edges": np.zeros(n, np.int32),
           "weight": np.zeros(n, np.int64), "obs": np.zeros(n, np.uint64), "status": np.zeros(n, np.int32)}
    outs = [dec.alloc(1) for _ in range(8)]
    for i in range(n):
        dec.decode_into(synd[i:i + 1], outs[i % 8])
        if i % 8 == 7 or i == n - 1:
            torch.cuda.synchronize()
            for j in range(i - i % 8, i + 1):
                o = outs[j % 8]
                res["edges"][j] = o.edges.cpu().numpy()[0]; res["n_edges"][j] = o.n_edges.cpu().numpy()[0]
                res["weight"][j] = o.weight.cpu().numpy()[0]; res["obs"][j] = o.obs.cpu().numpy().view(np.uint64)[0]
                res["status"][j] = o.status.cpu().numpy()[0]
    dec.close(); G.close()
    bad = compare(g, s.syndromes, res, range(n))
    say(f"d5 one launch per shot: {n} shots, {len(bad)} differ")
    assert not bad, bad[:5]


def test_d21_timelike_q02_partition_mode_every_shot():
    """Decoding weights for timelike flips at q = 0.2 against spatial
    p = 0.005 (d=21, 21 rounds): the level-1 clustering search needs paths of
    up to seven edges (the generic walk with near lists).  The syndromes are
    sampled at p = q = 0.005 on the same edges (at q = 0.2 itself about 40 %
    of the detectors fire, beyond every tier's capacity); 20,000 shots in one
    launch with the default partition-and-fuse decoder, every one equal to
    the oracle on the q = 0.2 weights."""
    g = synth.rotated_phenom_graph(21, 0.005, q=0.2)
    gs = synth.rotated_phenom_graph(21, 0.005)
    assert np.array_equal(g.u, gs.u) and np.array_equal(g.v, gs.v)
    s = synth.sample(gs, 20000, seed=170)
    say("d21 q=0.2 weights: decoding 20000 shots")
    res = gpu_decode(g, s.syndromes)
    _every_shot(g, s.syndromes, res, "d21 q=0.2 weights")
