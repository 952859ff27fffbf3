"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/rcpsp.h, and rejects malformed instances with the
documented status codes before touching the device."""
import os
import re

import pytest

from paper_1711_04556_amd import rcpsp, synth
from tests.conftest import ROOT


def declared_functions():
    with open(os.path.join(ROOT, "include", "rcpsp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rcpsp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = rcpsp.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_version_string():
    assert "gfx950" in rcpsp.version()


def test_potential_moves_closed_form():
    for N, d in [(3, 1), (12, 3), (32, 8), (122, 20), (302, 20), (10, 64)]:
        Lp = N - 2
        dd = min(d, Lp - 1)
        expect = dd * Lp - dd * (dd + 1) // 2 if Lp >= 2 else 0
        assert rcpsp.potential_moves(N, d) == expect


def _expect(inst, status, eval=rcpsp.EVAL_AUTO):
    with pytest.raises(rcpsp.RcpspError) as e:
        rcpsp.Instance(inst, eval=eval)
    assert e.value.status == status, str(e.value)


def _clone(inst, **kw):
    d = dict(n=inst.n, m=inst.m, duration=list(inst.duration), capacity=list(inst.capacity),
             request=list(inst.request), succ=[list(s) for s in inst.succ])
    d.update(kw)
    return synth.Instance(**d)


def test_rejects_nonzero_dummy_duration():
    t = synth.table1_instance()
    d = list(t.duration)
    d[-1] = 2
    _expect(_clone(t, duration=d), -4)


def test_rejects_request_above_capacity():
    t = synth.table1_instance()
    r = list(t.request)
    r[2] = 7
    _expect(_clone(t, request=r), -3)


def test_rejects_dummy_request():
    t = synth.table1_instance()
    r = list(t.request)
    r[0] = 1
    _expect(_clone(t, request=r), -4)


def test_rejects_cycle():
    t = synth.table1_instance()
    s = [list(x) for x in t.succ]
    s[7].append(4)          # 4 -> 7 -> 4
    _expect(_clone(t, succ=[sorted(x) for x in s]), -2)


def test_rejects_missing_source_arc():
    t = synth.table1_instance()
    s = [list(x) for x in t.succ]
    s[0] = [1]               # activity 2 loses its only predecessor
    _expect(_clone(t, succ=s), -4)


def test_rejects_missing_sink_arc():
    t = synth.table1_instance()
    s = [list(x) for x in t.succ]
    s[9] = []                # activity 9 loses its only successor
    _expect(_clone(t, succ=s), -4)


def test_rejects_out_of_range_successor():
    t = synth.table1_instance()
    s = [list(x) for x in t.succ]
    s[3] = [5, 12]
    _expect(_clone(t, succ=s), -1)


def test_rejects_horizon_too_large():
    t = synth.table1_instance()
    d = list(t.duration)
    d[1] = 40000
    _expect(_clone(t, duration=d), -9)


def test_rejects_too_many_resources():
    t = synth.table1_instance()
    _expect(_clone(t, m=17, capacity=[6] * 17, request=[0] * (12 * 17)), -9)
