"""Pins of the oracle's forward-backward improvement (the improvement of
every second initial solution, which the paper cites from Li and Willis).
Checked against what the mathematics fixes: schedules stay feasible
(eqs. 3-4), a justification pass never lengthens a schedule built by the
time-indexed serial SGS, the stopping rule makes the result a fixed point,
no result beats the brute-force optimum, and without resource conflicts
nothing changes."""
import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth
from tests.test_oracle_pins import brute_force_optimum, check_schedule

TIME, CAP = oracle.TIME, oracle.CAPACITY


def _reversed(inst):
    """The same project with every arc reversed (0 becomes the sink)."""
    succ = [[] for _ in range(inst.n)]
    for i in range(inst.n):
        for j in inst.succ[i]:
            succ[j].append(i)
    return synth.Instance(n=inst.n, m=inst.m, duration=inst.duration, capacity=inst.capacity,
                          request=inst.request, succ=[sorted(s) for s in succ], name=inst.name + "-rev")


def _by_desc(key, order):
    pos = {a: p for p, a in enumerate(order)}
    return sorted(range(len(order)), key=lambda a: (-key[a], -pos[a]))


def _instances():
    return [synth.generate(25, 4, 10, 0.5, rs=rs, seed=700 + k) for k, rs in enumerate((0.2, 0.3, 0.5))] + \
           [synth.generate(40, 2, 8, 0.75, rs=0.25, seed=710)]


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_fbi_feasible_never_worse_and_fixed_point(dec):
    for inst in _instances():
        orc = oracle.Oracle(inst)
        for s in range(6):
            W = synth.random_feasible_order(inst, 40 + s)
            c0 = orc.decode(W, dec)
            W2, c2 = orc.fbi(W, dec)
            assert orc.is_feasible_order(W2)
            c, start = orc.decode(W2, dec, starts=True)
            assert c == c2 <= c0
            assert check_schedule(inst, start) == c2
            if c2 == c0:
                assert W2 == list(W)          # nothing accepted unless it improved
            assert orc.fbi(W2, dec) == (W2, c2)   # a fixed point


def test_justification_passes_never_lengthen():
    """One backward pass (activities by decreasing finish time on the
    reversed project) and one forward pass (by decreasing backward finish):
    each schedule is at most as long as the one before (time-indexed SGS)."""
    improved = 0
    for inst in _instances():
        orc, rev = oracle.Oracle(inst), oracle.Oracle(_reversed(inst))
        d = inst.duration
        for s in range(6):
            W = synth.random_feasible_order(inst, 60 + s)
            c0, st = orc.decode(W, TIME, starts=True)
            B = _by_desc([st[a] + d[a] for a in range(inst.n)], W)
            cb, sb = rev.decode(B, TIME, starts=True)
            assert cb <= c0
            F = _by_desc([sb[a] + d[a] for a in range(inst.n)], B)
            assert orc.is_feasible_order(F)
            cf = orc.decode(F, TIME)
            assert cf <= cb
            _, c2 = orc.fbi(W, TIME)
            assert c2 <= cf
            improved += c2 < c0
    assert improved > 0   # the improvement does something on these projects


def test_fbi_without_resource_conflicts_is_identity():
    for k in range(3):
        base = synth.generate(20, 3, 9, 0.5, rs=0.5, seed=720 + k)
        big = [sum(base.request[i * base.m + r] for i in range(base.n)) for r in range(base.m)]
        inst = synth.Instance(n=base.n, m=base.m, duration=base.duration, capacity=big, request=base.request,
                              succ=base.succ)
        orc = oracle.Oracle(inst)
        W = synth.random_feasible_order(inst, 5 + k)
        for dec in (TIME, CAP):
            assert orc.fbi(W, dec) == (list(W), orc.critical_path)


@pytest.mark.parametrize("idx", range(4))
def test_fbi_not_below_optimum(idx):
    inst = synth.random_tiny(80 + idx, n_real=5)
    opt = brute_force_optimum(inst)
    orc = oracle.Oracle(inst)
    for s in range(4):
        W = synth.random_feasible_order(inst, s)
        assert orc.fbi(W, TIME)[1] >= opt


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_search_improves_every_second_initial_solution(dec):
    """With the improvement on, independent searches of even index follow the
    same trajectory as without it; searches of odd index start from the
    improved order of their initial solution."""
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=730)
    orc = oracle.Oracle(inst)
    kw = dict(searches=4, decoder=dec, seed=3)
    a = orc.tabu_search(8, 30, 12, **kw)
    b = orc.tabu_search(8, 30, 12, fbi=True, **kw)
    for s in (0, 2):
        assert np.array_equal(a["trajectory"][s], b["trajectory"][s])
    for s in (1, 3):
        W, c = orc.fbi(orc.initial_order(3, s), dec)
        assert b["best_makespan"][s] <= c
        if b["trajectory"][s][0][0] >= 0:
            assert b["trajectory"][s][0][3] <= c
