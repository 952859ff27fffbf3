"""Oracle pins for the decoder schedule of periodic re-selection (the
experimental set-up of Section 7 re-times the decoders every 1000
iterations).  The two decoders are different functions (the time-indexed
serial schedule back-fills, the capacity-indexed one does not), so a
schedule changes the search; these tests fix what it must do:

* a constant schedule is the plain search with that decoder;
* a switching schedule, replayed move by move from the initial orders with
  per-move decodes, takes in every iteration the lexicographically smallest
  admissible (C', u, v) of the neighbourhood decoded with that iteration's
  decoder (tabu list of Alg. 3, aspiration by the search's best);
* with a working set, results stay consistent (every best and record
  makespan is its order's makespan under one of the decoders).  Which
  decoder decodes a diversified read (the one of the iteration that
  completes it) is a convention shared with the device path and is not
  pinned here beyond a constant schedule.
"""
import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth

TIME, CAP = 1, 2


def _inst():
    # an instance whose two decoders lead the search apart
    return synth.generate(30, 4, 10, 0.5, rs=0.4, seed=1201)


@pytest.mark.parametrize("elite", [0, 4])
@pytest.mark.parametrize("dec", [TIME, CAP])
def test_constant_schedule_is_the_plain_search(dec, elite):
    orc = oracle.Oracle(_inst())
    kw = dict(searches=5, elite=elite, phi_max=1, phi_steps=3, seed=9)
    a = orc.tabu_search(6, 12, 30, decoder=dec, **kw)
    c = orc.tabu_search(6, 12, 30, decoder=dec, decoder_of_iteration=[dec] * 30, **kw)
    for key in ("best_makespan", "iterations_done", "evaluations", "best_order", "trajectory",
                "elite_makespan", "elite_order"):
        assert np.array_equal(a[key], c[key]), key


def _replay(orc, inst, sched, delta, tl, seed, b, iters, traj, c0_dec):
    n = orc.n
    w = orc.initial_order(seed, b)
    c_best = orc.decode(w, c0_dec)
    ring = [None] * tl
    widx = 0
    tabu = set()
    for it in range(iters):
        if traj[it, 0] < 0:
            break
        dec = sched[it]
        best = None
        fallback = None
        for u in range(1, n - 1):
            for v in range(u + 1, min(n - 2, u + delta) + 1):
                if not orc.move_feasible(w, u, v):
                    continue
                x = list(w)
                x[u], x[v] = x[v], x[u]
                key = (orc.decode(x, dec), u, v)
                if fallback is None or key < fallback:
                    fallback = key
                if ((u, v) not in tabu or key[0] < c_best) and (best is None or key < best):
                    best = key
        pick = best if best is not None else fallback
        assert (traj[it, 2], traj[it, 0], traj[it, 1]) == pick, (b, it)   # rows are (u, v, C', C_best)
        c, u, v = pick
        w[u], w[v] = w[v], w[u]
        old = ring[widx]
        if old is not None:
            tabu.discard(old)
        ring[widx] = (u, v)
        tabu.add((u, v))
        widx = (widx + 1) % tl
        c_best = min(c_best, c)
        assert traj[it, 3] == c_best


def test_switching_schedule_replays_move_by_move():
    inst = _inst()
    orc = oracle.Oracle(inst)
    iters, delta, tl, seed, B = 36, 6, 12, 9, 3
    sched = [TIME] * 5 + [CAP] * 7 + [TIME] * 10 + [CAP] * 14
    r = orc.tabu_search(delta, tl, iters, searches=B, decoder=TIME, seed=seed, decoder_of_iteration=sched)
    plain = orc.tabu_search(delta, tl, iters, searches=B, decoder=TIME, seed=seed)
    assert not np.array_equal(r["trajectory"], plain["trajectory"])   # the schedule matters here
    for b in range(B):
        _replay(orc, inst, sched, delta, tl, seed, b, iters, r["trajectory"][b], TIME)
    # the set-up decoder decodes the initial orders only: C_best starts from it
    r2 = orc.tabu_search(delta, tl, iters, searches=B, decoder=CAP, seed=seed, decoder_of_iteration=sched)
    for b in range(B):
        _replay(orc, inst, sched, delta, tl, seed, b, iters, r2["trajectory"][b], CAP)


def test_working_set_schedule_results_are_consistent():
    orc = oracle.Oracle(_inst())
    iters = 40
    kw = dict(searches=6, elite=3, phi_max=0, phi_steps=4, seed=5)
    sched = [TIME if (it // 4) % 2 == 0 else CAP for it in range(iters)]
    r = orc.tabu_search(6, 12, iters, decoder=TIME, decoder_of_iteration=sched, **kw)
    t = orc.tabu_search(6, 12, iters, decoder=TIME, **kw)
    assert not np.array_equal(r["trajectory"], t["trajectory"])   # the schedule matters here
    # every best and working-set makespan is its order's makespan under one
    # of the two decoders (which one depends on the iteration that reached it)
    for k in range(kw["elite"]):
        w = r["elite_order"][k].tolist()
        assert orc.is_feasible_order(w)
        assert r["elite_makespan"][k] in (orc.decode(w, TIME), orc.decode(w, CAP))
    for b in range(kw["searches"]):
        w = r["best_order"][b].tolist()
        assert r["best_makespan"][b] in (orc.decode(w, TIME), orc.decode(w, CAP))
        done = r["trajectory"][b, :, 3]
        done = done[done >= 0]
        assert (np.diff(done) <= 0).all() and done[-1] == r["best_makespan"][b]
