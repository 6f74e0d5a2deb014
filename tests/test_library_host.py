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
