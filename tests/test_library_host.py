"""CPU-only checks of the C-ABI library: it loads, exports every declared
symbol, and its host-side schedule equals the oracle's exact schedule."""
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "psb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(psb_[a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("psb_graph_create", "psb_decoder_create", "psb_decode_batch", "psb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2609_12262_amd as psb
    L = psb.lib()
    for n in _declared_functions():
        assert hasattr(L, n), f"{n} not exported"


@pytest.mark.parametrize("w", [2710, 2972, 3536, 17, 3])
def test_library_schedule_equals_oracle(w):
    import paper_2609_12262_amd as psb
    diam = 10 ** 12
    d, b, fin = psb.schedule_levels(w, diam)
    od, ob, _ = oracle.schedule(w, levels=len(d))
    assert d == od and b == ob
    assert fin[-1] == 1 and all(f == 0 for f in fin[:-1])
    assert b[-1] >= diam and (len(b) == 1 or b[-2] < diam)


def test_library_schedule_tiebroken_units():
    """Same schedule in tie-broken units (w_max ~ 2^76) as the oracle's Fractions."""
    import paper_2609_12262_amd as psb
    wmax = (2 * 1355 << 64) + 2 * 123456789
    d, b, fin = psb.schedule_levels(wmax, 10 ** 30)
    od, ob, _ = oracle.schedule(wmax, levels=len(d))
    assert d == od and b == ob


def test_library_rejects_bad_schedule_arguments():
    import paper_2609_12262_amd as psb
    with pytest.raises(psb.PsbError):
        psb.schedule_levels(100, 1000, q=(2, 1))
    with pytest.raises(psb.PsbError):
        psb.schedule_levels(0, 1000)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and a
    message, before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _create_raw(n, u, v, w, obs=None):
    """psb_graph_create on raw arrays; returns (code, message, handle)."""
    import ctypes
    import numpy as np
    import paper_2609_12262_amd as psb
    u = np.ascontiguousarray(u, np.int32); v = np.ascontiguousarray(v, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    obs = np.zeros(len(u), np.uint64) if obs is None else np.ascontiguousarray(obs, np.uint64)
    desc = psb._GraphDesc(n, len(u), u.ctypes.data, v.ctypes.data, w.ctypes.data, obs.ctypes.data)
    h = ctypes.c_void_p()
    rc = psb.lib().psb_graph_create(ctypes.byref(desc), ctypes.byref(h))
    return rc, psb.lib().psb_last_error().decode(), h


@pytest.mark.parametrize("case,n,u,v,w,why", [
    ("zero weight", 3, [0, 1], [1, 2], [5, 0], "non-positive weight"),
    ("negative weight", 3, [0, 1], [1, -1], [5, -3], "non-positive weight"),
    ("u out of range", 3, [0, 3], [1, 2], [5, 5], "out of range"),
    ("negative u", 3, [-1, 1], [1, 2], [5, 5], "out of range"),
    ("v below the boundary code", 3, [0, 1], [1, -2], [5, 5], "out of range"),
    ("v out of range", 3, [0, 1], [1, 7], [5, 5], "out of range"),
    ("self loop", 3, [0, 1], [1, 1], [5, 5], "self loop"),
    ("no detectors", 0, [], [], [], "num_detectors"),
    ("degree above 16", 2, [0] * 17, [1] * 17, [3] * 17, "degree"),
])
def test_graph_create_rejects_malformed_graphs(case, n, u, v, w, why):
    """The decoding task needs positive weights on a graph whose edges join
    distinct detectors or a detector and its own boundary vertex (Results,
    "Decoding task"): anything else is refused with PSB_E_INVALID and a
    message, before any device work."""
    import paper_2609_12262_amd as psb
    rc, msg, h = _create_raw(n, u, v, w)
    assert rc == psb.PSB_E_INVALID, case
    assert why in msg, (case, msg)
    assert not h.value


def test_null_arguments_are_refused():
    import ctypes
    import paper_2609_12262_amd as psb
    L = psb.lib()
    h = ctypes.c_void_p()
    assert L.psb_graph_create(None, ctypes.byref(h)) == psb.PSB_E_INVALID
    assert L.psb_decoder_create(None, None, ctypes.byref(h)) == psb.PSB_E_INVALID
    assert L.psb_decode_batch(None, None, ctypes.c_int64(1), None, None, None, None, None, None, None, None,
                              None) == psb.PSB_E_INVALID
    assert L.psb_batch_graph_launch(None, None) == psb.PSB_E_INVALID
    assert L.psb_server_submit(None, 0, None, None, None) == psb.PSB_E_INVALID
