"""GPU: periodic decoder re-selection (rcpsp_tabu_search_reselect, C ABI).
The decoder is re-chosen by timing, so the run is checked per segment: the
CPU oracle replays it with the logged decoder of every iteration (set-up
decodes with the instance's decoder) and must give exactly the same
results; the log must cover the iterations in order, probe both decoders at
the start of every period and continue with the faster one."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth

pytestmark = pytest.mark.gpu

TIME, CAP = 1, 2


@pytest.fixture(scope="module")
def rc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_04556_amd import rcpsp
    rcpsp.lib()
    return rcpsp


def _schedule(segs, iters):
    sched = [0] * iters
    for s in segs:
        for it in range(s["first_iteration"], s["first_iteration"] + s["iterations"]):
            sched[it] = s["eval"]
    assert 0 not in sched
    return sched


def _check_log(segs, iters, period, probe, decoders):
    it = 0
    while it < iters:
        end = min(iters, it + period)
        seg = []
        while segs and segs[0]["first_iteration"] < end:
            seg.append(segs.pop(0))
        assert seg and seg[0]["first_iteration"] == it
        for a, b in zip(seg, seg[1:]):
            assert b["first_iteration"] == a["first_iteration"] + a["iterations"]
        assert seg[-1]["first_iteration"] + seg[-1]["iterations"] == end
        probes = [s for s in seg if s["probe"]]
        runs = [s for s in seg if not s["probe"]]
        if len(decoders) > 1:
            assert [s["eval"] for s in probes] == decoders[:len(probes)]
            assert all(s["iterations"] == min(probe, end - s["first_iteration"]) for s in probes)
            assert len(runs) <= 1
            if runs and len(probes) == 2:
                t = {s["eval"]: s["ms_per_iteration"] for s in probes}
                want = CAP if t[CAP] < t[TIME] else TIME
                assert runs[0]["eval"] == want
        else:
            assert not probes and len(runs) == 1 and runs[0]["eval"] == decoders[0]
        assert all(s["ms_per_iteration"] > 0 for s in seg)
        it = end
    assert not segs


@pytest.mark.parametrize("elite", [0, 4])
def test_reselection_matches_oracle_replay(rc, elite):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.4, seed=1201)
    gi = rc.Instance(inst)
    iters, period, probe = 45, 12, 3
    kw = dict(swap_range=8, tabu_len=20, iterations=iters, searches=6, elite=elite, phi_max=2, phi_steps=4,
              seed=17)
    res, segs = rc.tabu_search_reselect(gi, period, probe, **kw)
    o = oracle.Oracle(inst).tabu_search(8, 20, iters, searches=6, elite=elite, phi_max=2, phi_steps=4,
                                        decoder=gi.info["eval"], seed=17, decoder_of_iteration=_schedule(segs, iters))
    for key in ("best_makespan", "iterations_done", "evaluations", "best_order", "trajectory"):
        assert np.array_equal(res[key], o[key]), key
    if elite:
        assert np.array_equal(res["elite_makespan"], o["elite_makespan"])
        assert np.array_equal(res["elite_order"], o["elite_order"])
    assert res["global_best"] == min(o["best_makespan"].min(), o["elite_makespan"].min() if elite else 1 << 30)
    _check_log(list(segs), iters, period, probe, [TIME, CAP])


def test_reselection_follows_a_switch(rc):
    """Probes of three iterations in every period of six: both decoders run
    in every period, whichever is faster, so the replay always covers a
    switch."""
    inst = synth.generate(30, 4, 10, 0.5, rs=0.4, seed=1201)
    gi = rc.Instance(inst)
    iters = 30
    kw = dict(swap_range=8, tabu_len=20, iterations=iters, searches=4, elite=3, phi_max=0, phi_steps=4, seed=23)
    res, segs = rc.tabu_search_reselect(gi, 6, 3, **kw)
    sched = _schedule(segs, iters)
    assert set(sched) == {TIME, CAP}
    o = oracle.Oracle(inst).tabu_search(8, 20, iters, searches=4, elite=3, phi_max=0, phi_steps=4,
                                        decoder=gi.info["eval"], seed=23, decoder_of_iteration=sched)
    for key in ("best_makespan", "iterations_done", "evaluations", "best_order", "trajectory", "elite_makespan",
                "elite_order"):
        assert np.array_equal(res[key], o[key]), key
    _check_log(list(segs), iters, 6, 3, [TIME, CAP])


def test_reselection_with_one_decoder_that_fits(rc):
    # five resources (two dwords per time unit), durations up to 200: one
    # time-indexed profile of the ~25,000-unit horizon needs ~200 KB, more
    # than LDS holds; the capacity-indexed layout fits
    inst = synth.generate(250, 5, 200, 0.5, rs=0.5, seed=1202)
    gi = rc.Instance(inst)
    assert gi.info["horizon"] > 21000 and gi.info["eval"] == CAP
    iters, period = 7, 4
    kw = dict(swap_range=6, tabu_len=10, iterations=iters, searches=2, seed=3)
    res, segs = rc.tabu_search_reselect(gi, period, 1, **kw)
    o = oracle.Oracle(inst).tabu_search(6, 10, iters, searches=2, decoder=CAP, seed=3,
                                        decoder_of_iteration=_schedule(segs, iters))
    for key in ("best_makespan", "iterations_done", "evaluations", "best_order", "trajectory"):
        assert np.array_equal(res[key], o[key]), key
    _check_log(list(segs), iters, period, 1, [CAP])


def test_reselection_arguments(rc):
    inst = synth.generate(20, 2, 6, 0.5, rs=0.5, seed=1203)
    gi = rc.Instance(inst)
    L = rc.lib()
    p = rc.search_params(swap_range=6, tabu_len=8, iterations=10, searches=2, seed=1)
    res = rc.rcpsp_search_result()
    n = ctypes.c_int32(-1)
    for period, probe in ((4, 0), (3, 2)):
        st = L.rcpsp_tabu_search_reselect(gi.h, ctypes.byref(p), period, probe, ctypes.byref(res), None, 0,
                                          ctypes.byref(n), None)
        assert st == -1
    q = rc.search_params(swap_range=6, tabu_len=8, iterations=10, searches=2, seed=1, eval=TIME)
    assert L.rcpsp_tabu_search_reselect(gi.h, ctypes.byref(q), 4, 1, ctypes.byref(res), None, 0,
                                        ctypes.byref(n), None) == -1
    # a log too short: results complete, RCPSP_E_BUFFER, the number of segments reported
    best = np.zeros(2, np.int32)
    res = rc.rcpsp_search_result()
    res.best_makespan = best.ctypes.data
    log = (rc.rcpsp_decoder_segment * 2)()
    st = L.rcpsp_tabu_search_reselect(gi.h, ctypes.byref(p), 4, 1, ctypes.byref(res), log, 2, ctypes.byref(n),
                                      None)
    assert st == -6 and n.value == 8   # three periods: 3 + 3 + 2 segments
    full, _ = rc.tabu_search_reselect(gi, 4, 1, swap_range=6, tabu_len=8, iterations=10, searches=2, seed=1)
    assert np.array_equal(best, full["best_makespan"])
