"""GPU: captured batches (HIP graph replay) and the autotuner's candidate
configurations, through the C ABI.  Exact comparisons: every output is an
integer."""
import numpy as np
import pytest

import synth
from gpu_helpers import SEED, compare, gpu_decode, say

pytestmark = pytest.mark.gpu

KEYS = ("edges", "n_edges", "weight", "obs", "status")


def _host(out):
    h = {k: getattr(out, k).cpu().numpy() for k in KEYS}
    # entries past n_edges in a row are unspecified (left from earlier launches)
    h["edges"] = np.where(np.arange(h["edges"].shape[1])[None, :] < h["n_edges"][:, None], h["edges"], -1)
    return h


def test_batch_graph_replays_equal_eager():
    """A captured d=11 batch replayed 6 times over 3 refilled syndrome sets,
    with eager decodes and other device work between replays: every replay
    equals the eager decode of the same set, and the first equals the oracle."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(11, 0.003)
    sets = [synth.sample(g, 4096, seed=70 + k).syndromes for k in range(3)]
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=SEED)
    ref = psb.Decoder(G, tiebreak_seed=SEED)
    S = torch.from_numpy(sets[0]).cuda()
    out = dec.alloc(4096)
    bg = dec.capture(S, out)
    say("batch graph captured")
    junk = torch.arange(1 << 22, device="cuda", dtype=torch.int64)
    for r in range(6):
        k = r % 3
        S.copy_(torch.from_numpy(sets[k]))
        bg.launch()
        torch.cuda.synchronize()
        got = _host(out)
        e = ref.decode(torch.from_numpy(sets[k]).cuda())
        torch.cuda.synchronize()
        want = _host(e)
        for key in KEYS:
            assert np.array_equal(got[key], want[key]), (r, key)
        if r == 0:
            res = dict(got, obs=got["obs"].view(np.uint64))
            bad = compare(g, sets[0], res, range(0, 4096, 16))
            assert not bad, bad[:5]
        junk.add_(int(junk[r].item()) + 1)          # unrelated eager work between replays
        say(f"replay {r} equal")
    bg.close(); dec.close(); ref.close(); G.close()


def test_captured_graph_pins_the_overflow_list():
    """While a captured batch graph of a decoder exists, nothing may move the
    overflow list its kernel arguments hold: a larger batch, a larger reserve
    and a second capture for more shots are refused with an error before
    anything is launched.  After the graph is destroyed they succeed."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(9, 0.005)
    small = torch.from_numpy(synth.sample(g, 256, seed=81).syndromes).cuda()
    big_np = synth.sample(g, 1024, seed=82).syndromes
    big = torch.from_numpy(big_np).cuda()
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=SEED)
    out = dec.alloc(256)
    bg = dec.capture(small, out)
    out_big = dec.alloc(1024)
    with pytest.raises(psb.PsbError):
        dec.decode_into(big, out_big)
    with pytest.raises(psb.PsbError):
        dec.reserve(1024)
    with pytest.raises(psb.PsbError):
        dec.capture(big, out_big)
    bg.launch()
    torch.cuda.synchronize()
    got = _host(out)
    eager = _host(dec.decode(small))
    torch.cuda.synchronize()
    for key in KEYS:
        assert np.array_equal(got[key], eager[key]), key
    bg.close()
    dec.reserve(1024)
    res = _host(dec.decode_into(big, out_big))
    torch.cuda.synchronize()
    res["obs"] = res["obs"].view(np.uint64)
    bad = compare(g, big_np, res, range(0, 1024, 4))
    assert not bad, bad[:5]
    dec.close(); G.close()


def test_autotune_candidates_agree_and_best_matches_oracle():
    """d=21, p=0.007 (some shots exceed the default first-tier state): every
    candidate that fits decodes the sample to the same weights and
    observables (checked inside psb_autotune); the chosen configuration
    decodes a fresh batch equal to the oracle on sampled shots."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(21, 0.007)
    s = synth.sample(g, 4096, seed=80)
    G = psb.Graph.from_synth(g)
    best, table = psb.autotune(G, torch.from_numpy(s.syndromes).cuda(), reps=1, tiebreak_seed=SEED)
    say(f"autotune best {best}")
    ok = [t for t in table if t["status"] == 0]
    assert ok and all(t["ms"] > 0 for t in ok)
    assert min(t["ms"] for t in ok) == [t for t in table if all(t[k] == best[k] for k in best)][0]["ms"]
    G.close()
    s2 = synth.sample(g, 3000, seed=81)
    kw = {k: best[k] for k in ("fast_max_nodes", "fast_max_regions", "first_tier", "fast_lds_state")}
    res = gpu_decode(g, s2.syndromes, **kw)
    bad = compare(g, s2.syndromes, res, range(0, 3000, 20))
    assert not bad, bad[:5]


@pytest.mark.parametrize("q", [(1, 4), (1, 3)])
def test_schedule_ratio_does_not_change_result(q):
    """The partition-and-fuse result is the MWEM for any admissible schedule
    ratio q: d=13, p=0.005, every shot equals the oracle."""
    import torch
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(13, 0.005)
    s = synth.sample(g, 3000, seed=90)
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=SEED, q=q)
    out = dec.decode(torch.from_numpy(s.syndromes).cuda())
    torch.cuda.synchronize()
    res = _host(out)
    res["obs"] = res["obs"].view(np.uint64)
    dec.close(); G.close()
    bad = compare(g, s.syndromes, res, range(3000))
    assert not bad, bad[:5]


@pytest.mark.parametrize("lds_state,caps", [(2, (0, 0)), (3, (0, 0)), (3, (1024, 768)), (4, (0, 0)),
                                            (4, (2048, 1024))])
def test_first_tier_state_placement_parity(lds_state, caps):
    """Where the first tier keeps its per-shot state (LDS, workspace, or all
    of it in the workspace with no LDS) does not change results: d=13,
    p=0.005, every shot equals the oracle."""
    g = synth.rotated_phenom_graph(13, 0.005)
    s = synth.sample(g, 3000, seed=91)
    res = gpu_decode(g, s.syndromes, fast_lds_state=lds_state, fast_max_nodes=caps[0], fast_max_regions=caps[1],
                     want_overflow=True)
    say(f"lds_state={lds_state} caps={caps}: {res['n_overflow']} shots in the overflow tier")
    bad = compare(g, s.syndromes, res, range(3000))
    assert not bad, bad[:5]


def _accounted(g, syndromes, **kw):
    import torch
    import paper_2609_12262_amd as psb
    G = psb.Graph.from_synth(g)
    dec = psb.Decoder(G, tiebreak_seed=SEED, event_accounting=1, **kw)
    out = dec.decode(torch.from_numpy(syndromes).cuda(), levels=True, stats=True)
    torch.cuda.synchronize()
    res = _host(out)
    res["obs"] = res["obs"].view(np.uint64)
    res["stats"] = out.stats.cpu().numpy()
    res["levels"] = out.levels.cpu().numpy()
    dec.close(); G.close()
    return res


def test_event_accounting_properties():
    """Per-cluster event accounting (the parallel event count E_ideal of
    hierarchical execution): results equal those without accounting; E_ideal
    is at most the applied events, positive exactly when the shot has events;
    the processing clusters and highest level equal the oracle's clustering
    (one final cluster for the events left at the final level)."""
    import oracle
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(11, 0.005)
    s = synth.sample(g, 2000, seed=95)
    acc = _accounted(g, s.syndromes)
    plain = gpu_decode(g, s.syndromes)
    for key in ("n_edges", "weight", "obs", "status"):
        assert np.array_equal(acc[key], plain[key]), key
    st = acc["stats"]
    nd = np.array([len(synth.defects_of(r, g.num_detectors)) for r in s.syndromes])
    assert (st[:, 9] <= st[:, 8]).all()
    assert ((st[:, 9] > 0) == (nd > 0)).all()
    assert ((st[:, 10] > 0) == (nd > 0)).all()
    og = oracle.Graph(g, SEED)
    dec = psb.Decoder(psb.Graph.from_synth(g), tiebreak_seed=SEED)
    d_k, b_k, fin = dec.levels()
    kf = fin.index(1) + 1
    od, ob, _ = oracle.schedule(max(og.tiebroken_weights()), levels=max(len(d_k), 4))
    checked = 0
    for i in range(0, 2000, 7):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        if len(dd) == 0:
            continue
        D, _ = og.defect_distances(dd)
        lv, comps = oracle.cluster_levels(D, og.boundary_table(dd), od, ob, components=True)
        n_cl = sum(1 for k, _ in comps if k < kf) + (1 if any(x >= kf or x == 0 for x in lv) else 0)
        top = max(min(x, kf) if x else kf for x in lv)
        assert st[i, 10] == n_cl, (i, st[i, 10], n_cl)
        assert st[i, 11] == top, (i, st[i, 11], top)
        checked += 1
    assert checked > 100


def test_event_accounting_global_mode_and_lane_tier():
    """Global sparse blossom is one cluster: E_ideal equals the applied
    events.  The lane tier processes the same events: same counts."""
    g = synth.rotated_phenom_graph(9, 0.005)
    s = synth.sample(g, 1500, seed=96)
    glob = _accounted(g, s.syndromes, mode=1)
    assert np.array_equal(glob["stats"][:, 9], glob["stats"][:, 8])
    nd = np.array([len(synth.defects_of(r, g.num_detectors)) for r in s.syndromes])
    assert ((glob["stats"][:, 10] == 1) == (nd > 0)).all()
    wave = _accounted(g, s.syndromes)
    lane = _accounted(g, s.syndromes, first_tier=1)
    for q in (8, 9, 10, 11):
        assert np.array_equal(wave["stats"][:, q], lane["stats"][:, q]), q
    bad = compare(g, s.syndromes, wave, range(0, 1500, 5))
    assert not bad, bad[:5]


@pytest.mark.parametrize("d,rounds,W,C,p", [(5, 12, 6, 3, 0.01), (9, 30, 10, 5, 0.005), (11, 44, 22, 11, 0.003)])
def test_sliding_window_equals_oracle(d, rounds, W, C, p):
    """Sliding-window decoding (windows of W layers committing C): every
    shot's committed weight and observable equal the oracle's windowed
    decode, and every detection event is resolved."""
    import torch
    import oracle
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(d, p, rounds=rounds)
    L = (d * d - 1) // 2
    s = synth.sample(g, 400, seed=100 + d)
    plan = psb.WindowPlan(g, L, W, C, tiebreak_seed=SEED)
    out = plan.decode(torch.from_numpy(s.syndromes).cuda())
    torch.cuda.synchronize()
    say(f"window d={d} rounds={rounds}: {plan.n_windows} windows, {plan.n_shapes} window graphs")
    st = out["status"].cpu().numpy(); wt = out["weight"].cpu().numpy(); ob = out["obs"].cpu().numpy().view(np.uint64)
    plan.close()
    assert (st == 0).all(), np.bincount(st)
    sch = oracle.window_schedule(g, L, W, C)
    gs = [oracle.Graph(wg, SEED) for _, wg, _, _ in sch]
    for i in range(0, 400, 2):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        w, o, ok = oracle.window_decode(g, sch, gs, L, dd)
        assert ok and (int(wt[i]), int(ob[i])) == (w, o), (i, int(wt[i]), w, int(ob[i]), o)


def test_circuit_x_graph_autotune_windows_and_accounting():
    """The circuit-level X-fault graph (non-uniform weights, diagonal
    spacetime edges) through the autotuner (its candidates agree), sliding
    windows (equal to the oracle's windowed decode) and event accounting
    (E_ideal at most the applied events, results unchanged)."""
    import torch
    import oracle
    import paper_2609_12262_amd as psb
    g = synth.rotated_circuit_x_graph(9, 0.002)
    s = synth.sample(g, 2000, seed=130)
    G = psb.Graph.from_synth(g)
    best, table = psb.autotune(G, torch.from_numpy(s.syndromes).cuda(), reps=1, tiebreak_seed=SEED)
    assert any(t["status"] == 0 for t in table)
    acc = _accounted(g, s.syndromes)
    plain = gpu_decode(g, s.syndromes, **{k: best[k] for k in ("fast_max_nodes", "fast_max_regions", "first_tier",
                                                               "fast_lds_state")})
    for key in ("n_edges", "weight", "obs", "status"):
        assert np.array_equal(acc[key], plain[key]), key
    assert (acc["stats"][:, 9] <= acc["stats"][:, 8]).all()
    bad = compare(g, s.syndromes, plain, range(0, 2000, 10))
    assert not bad, bad[:5]
    G.close()
    gw = synth.rotated_circuit_x_graph(7, 0.002, rounds=21)
    L = (7 * 7 - 1) // 2
    sw = synth.sample(gw, 300, seed=131)
    plan = psb.WindowPlan(gw, L, 8, 4, tiebreak_seed=SEED)
    out = plan.decode(torch.from_numpy(sw.syndromes).cuda())
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy(); wt = out["weight"].cpu().numpy(); ob = out["obs"].cpu().numpy().view(np.uint64)
    plan.close()
    assert (st == 0).all(), np.bincount(st)
    sch = oracle.window_schedule(gw, L, 8, 4)
    gs = [oracle.Graph(wg, SEED) for _, wg, _, _ in sch]
    for i in range(0, 300, 3):
        w, o, ok = oracle.window_decode(gw, sch, gs, L, synth.defects_of(sw.syndromes[i], gw.num_detectors))
        assert ok and (int(wt[i]), int(ob[i])) == (w, o), i


@pytest.mark.parametrize("model", ["uniform", "physical"])
def test_sliding_windows_on_circuit_noise_graphs(model):
    """Sliding windows over 21 rounds of the X-memory circuit-level graphs
    (diagonal edges between adjacent layers, degree up to 12): every stream
    resolves and equals the oracle's windowed decode."""
    import torch
    import oracle
    import paper_2609_12262_amd as psb
    g = synth.rotated_circuit_graph(7, 0.002, model, rounds=21)
    L = (7 * 7 - 1) // 2
    s = synth.sample(g, 300, seed=170)
    say(f"windows on circuit {model}: 300 streams")
    plan = psb.WindowPlan(g, L, 8, 4, tiebreak_seed=SEED)
    out = plan.decode(torch.from_numpy(s.syndromes).cuda())
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy(); wt = out["weight"].cpu().numpy(); ob = out["obs"].cpu().numpy().view(np.uint64)
    plan.close()
    assert (st == 0).all(), np.bincount(st)
    sch = oracle.window_schedule(g, L, 8, 4)
    gs = [oracle.Graph(wg, SEED) for _, wg, _, _ in sch]
    for i in range(0, 300, 3):
        w, o, ok = oracle.window_decode(g, sch, gs, L, synth.defects_of(s.syndromes[i], g.num_detectors))
        assert ok and (int(wt[i]), int(ob[i])) == (w, o), i


def test_complementary_gap_wide_weight_range():
    """A graph whose lightest edge is under a tenth of the heaviest (timelike
    flips at q=0.4) needs level-1 search paths deeper than the clustering
    kernel walks, so a partition-and-fuse decoder is refused; the
    complementary plan then takes its MWEM side from global sparse blossom
    and still equals the oracle."""
    import torch
    import oracle
    import paper_2609_12262_amd as psb
    g = synth.rotated_phenom_graph(5, 0.005, q=0.4)
    G = psb.Graph.from_synth(g)
    with pytest.raises(psb.PsbError, match="needs paths of more than"):
        psb.Decoder(G, tiebreak_seed=SEED)
    G.close()
    s = synth.sample(g, 1000, seed=180)
    plan = psb.ComplementaryPlan(g, 0, tiebreak_seed=SEED)
    out = plan.decode(torch.from_numpy(s.syndromes).cuda())
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy() for k, v in out.items()}
    plan.close()
    assert (h["status"] == 0).all(), np.bincount(h["status"])
    co = oracle.Complementary(g, 0, SEED)
    for i in range(0, 1000, 2):
        w0, w1 = co.weights(synth.defects_of(s.syndromes[i], g.num_detectors))
        assert (int(h["weight0"][i]), int(h["weight1"][i])) == (w0, w1), i


_LANE_TIER = dict(first_tier=1, fast_max_nodes=2048, fast_max_regions=4096, num_slots=4096)


@pytest.mark.parametrize("graph,d,p,n,step,opts", [
    ("phenom", 5, 0.01, 3000, 1, {}), ("phenom", 11, 0.005, 2000, 4, {}),
    ("phenom", 11, 0.005, 2000, 4, dict(fast_max_nodes=320, fast_max_regions=208)), ("circuit_x", 7, 0.002, 1500, 3, {}),
    ("phenom", 13, 0.005, 1000, 4, {}), ("phenom", 13, 0.005, 256, 4, _LANE_TIER),
    ("circuit_uniform", 9, 0.003, 1000, 5, {}), ("phenom", 21, 0.005, 512, 8, {})])
def test_complementary_gap_equals_oracle(graph, d, p, n, step, opts):
    """Complementary-gap decoding: both constrained minimum weights (hence the
    gap) equal the oracle's, the reported observable is the MWEM's, and the
    lighter side equals the MWEM weight.  By default the first tier holds the
    whole rewritten graph; one case asks for the library's usual first tier
    (with shots handed to the overflow tier), one for the lane tier."""
    import torch
    import oracle
    import paper_2609_12262_amd as psb
    g = {"phenom": lambda: synth.rotated_phenom_graph(d, p), "circuit_x": lambda: synth.rotated_circuit_x_graph(d, p),
         "circuit_uniform": lambda: synth.rotated_circuit_graph(d, p, "uniform")}[graph]()
    s = synth.sample(g, n, seed=140 + d)
    say(f"complementary {graph} d={d} opts={opts}: {n} shots")
    plan = psb.ComplementaryPlan(g, 0, tiebreak_seed=SEED, **opts)
    out = plan.decode(torch.from_numpy(s.syndromes).cuda())
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy() for k, v in out.items()}
    plan.close()
    assert (h["status"] == 0).all(), np.bincount(h["status"])
    co = oracle.Complementary(g, 0, SEED)
    og = oracle.Graph(g, SEED)
    for i in range(0, n, step):
        dd = synth.defects_of(s.syndromes[i], g.num_detectors)
        w0, w1 = co.weights(dd)
        r = og.mwem(dd)
        assert (int(h["weight0"][i]), int(h["weight1"][i])) == (w0, w1), (i, h["weight0"][i], h["weight1"][i], w0, w1)
        assert int(h["gap"][i]) == abs(w1 - w0)
        assert min(w0, w1) == r.weight
        if w0 != w1:
            assert int(h["obs"][i]) & 1 == int(r.obs) & 1
