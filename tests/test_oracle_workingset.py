"""Pins of the oracle's working-set protocol (Section 6.1, eq. 8) by an
independent move-by-move replay.

The paper's working set is lock-based and timing dependent; the library and
the oracle take a round-synchronous reading of it (readings 17-19 of the
design notes, stated again here so the replay can be checked by eye):

* after the initial orders, search b reads record b mod |F|; afterwards,
  after every iteration (or every `exchange_every` iterations) the searches
  whose exchange condition fired are taken in ascending id;
* the condition: the best solution since the last read improves on the
  read makespan, or more than I_assigned iterations passed since the read;
* a search first adds its iterations since the read to the record's IC;
  it writes its best solution since the read (with its current tabu list)
  to the record it read only if that beats both the makespan it read and
  the record's current makespan; a write resets IC and the read count;
* it then reads the next record (cyclically): the record's read count goes
  up, and once it exceeds phi_max the order is diversified by phi_steps
  swaps, each drawn uniformly (by index) from the feasible moves of the
  current order in canonical order with the search's own random stream
  2^32 + b, the tabu list untouched, and the order decoded again;
* eq. 8 gives the read its I_assigned from the record's makespan (before
  diversification), the working set's best at that moment and the record's
  IC, with I_block = the iteration allowance;
* aspiration in an iteration is the minimum of the search's best and the
  working set's best after the last round; a stopped search (no feasible
  move) takes part in no round; the run ends early once the working set
  holds a critical-path schedule.

The replay calls the oracle only for what is pinned elsewhere (the decoders,
move feasibility, initial orders, eq. 8's integer table) and never for any
part of the round; it then compares every trajectory row, and after every
round every record's order, makespan, IC and read count and every search's
slot, I_assigned, read makespan and makespans, with the oracle's own log.
"""
import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth

TIME, CAP = oracle.TIME, oracle.CAPACITY
INF = 2 ** 31 - 1


def _moves(orc, W, delta):
    n = len(W)
    return [(u, v) for u in range(1, n - 1) for v in range(u + 1, min(n - 2, u + delta) + 1)
            if orc.move_feasible(W, u, v)]


def _pick(orc, W, delta, dec, tabu, asp):
    """Lexicographically smallest (C', u, v) among admissible moves, else
    among all feasible ones; and the number of feasible moves decoded."""
    best = fallback = None
    moves = _moves(orc, W, delta)
    for u, v in moves:
        x = list(W)
        x[u], x[v] = x[v], x[u]
        key = (orc.decode(x, dec), u, v)
        if fallback is None or key < fallback:
            fallback = key
        if ((u, v) not in tabu or key[0] < asp) and (best is None or key < best):
            best = key
    return (best if best is not None else fallback), len(moves)


def replay(orc, dec, delta, tl, iters, B, NF, phi_max, phi_steps, seed, every=1, stats=None):
    n = orc.n
    cp = orc.critical_path
    stats = stats if stats is not None else {}
    for k in ("writes", "rejected_writes", "multi_writer_rounds", "imp_differs_from_cur", "diversified",
              "diversify_changed_c", "expiry_fired", "rounds"):
        stats.setdefault(k, 0)
    recs = []
    for k in range(NF):
        W = orc.initial_order(seed, k)
        recs.append(dict(W=W, C=orc.decode(W, dec), ring=[(0, 0)] * tl, widx=0, tabu=set(), IC=0, reads=0))
    S = [dict(W=None, C_cur=INF, C_best=INF, W_best=None, W_imp=None, C_imp=INF, C_read=INF, ring=None, widx=0,
              tabu=None, slot=(b - 1) % NF, it_read=0, I_assigned=0, fired=True, stopped=False, it_done=0,
              evals=0, rng=synth.Stream(seed, 2 ** 32 + b)) for b in range(B)]
    traj = np.full((B, iters, 4), -1, np.int32)
    log = []

    def read(s, k):
        R = recs[k]
        R["reads"] += 1
        s["W"], s["C_cur"], s["C_read"] = list(R["W"]), R["C"], R["C"]
        s["ring"], s["widx"], s["tabu"] = list(R["ring"]), R["widx"], set(R["tabu"])
        if R["reads"] > phi_max:
            stats["diversified"] += 1
            for _ in range(phi_steps):
                mv = _moves(orc, s["W"], delta)
                if not mv:
                    break
                u, v = mv[s["rng"].below(len(mv))]
                s["W"][u], s["W"][v] = s["W"][v], s["W"][u]
            s["C_cur"] = orc.decode(s["W"], dec)
            stats["diversify_changed_c"] += int(s["C_cur"] != R["C"])
        s["W_imp"], s["C_imp"] = list(s["W"]), s["C_cur"]
        if s["C_cur"] < s["C_best"]:
            s["C_best"], s["W_best"] = s["C_cur"], list(s["W"])
        s["it_read"] = 0
        s["I_assigned"] = oracle.iterations_assigned(iters, R["C"], min(r["C"] for r in recs), R["IC"])
        s["slot"] = k

    def exchange():
        written = {}
        for s in S:
            if not s["fired"] or s["stopped"]:
                continue
            s["fired"] = False
            k = s["slot"]
            R = recs[k]
            R["IC"] += s["it_read"]
            if s["C_imp"] < s["C_read"]:
                if s["C_imp"] < R["C"]:
                    stats["writes"] += 1
                    stats["imp_differs_from_cur"] += int(s["W_imp"] != s["W"])
                    written[k] = written.get(k, 0) + 1
                    R.update(W=list(s["W_imp"]), C=s["C_imp"], ring=list(s["ring"]), widx=s["widx"],
                             tabu=set(s["tabu"]), IC=0, reads=0)
                else:
                    stats["rejected_writes"] += 1
            else:
                stats["expiry_fired"] += 1
            read(s, (k + 1) % NF)
        stats["multi_writer_rounds"] += int(any(c > 1 for c in written.values()))
        stats["rounds"] += 1
        log.append(dict(C=[r["C"] for r in recs], IC=[r["IC"] for r in recs], reads=[r["reads"] for r in recs],
                        W=[list(r["W"]) for r in recs], slot=[s["slot"] for s in S],
                        I_assigned=[s["I_assigned"] for s in S], C_read=[s["C_read"] for s in S],
                        C_cur=[s["C_cur"] for s in S], C_best=[s["C_best"] for s in S]))

    exchange()
    gstop = min(r["C"] for r in recs) == cp
    for it in range(iters):
        if gstop:
            break
        cstar = min(r["C"] for r in recs)
        for b, s in enumerate(S):
            if s["stopped"]:
                continue
            pick, nfeas = _pick(orc, s["W"], delta, dec, s["tabu"], min(s["C_best"], cstar))
            if nfeas == 0:
                s["stopped"] = True
                continue
            c, u, v = pick
            s["evals"] += nfeas
            s["W"][u], s["W"][v] = s["W"][v], s["W"][u]
            # Alg. 3: the oldest entry leaves the ring (and the cache), (u, v) enters
            s["tabu"].discard(s["ring"][s["widx"]])
            s["ring"][s["widx"]] = (u, v)
            s["tabu"].add((u, v))
            s["widx"] = (s["widx"] + 1) % tl
            s["C_cur"] = c
            if c < s["C_best"]:
                s["C_best"], s["W_best"] = c, list(s["W"])
            traj[b, it] = (u, v, c, s["C_best"])
            s["it_done"] += 1
            s["it_read"] += 1
            if c < s["C_imp"]:
                s["C_imp"], s["W_imp"] = c, list(s["W"])
            s["fired"] = s["C_imp"] < s["C_read"] or s["it_read"] > s["I_assigned"]
        if it < iters - 1 and (it + 1) % every == 0:
            exchange()
            gstop = min(r["C"] for r in recs) == cp
    return dict(trajectory=traj, best_makespan=[s["C_best"] for s in S], best_order=[s["W_best"] for s in S],
                iterations_done=[s["it_done"] for s in S], evaluations=[s["evals"] for s in S],
                elite_makespan=[r["C"] for r in recs], elite_order=[r["W"] for r in recs], rounds=log)


CONFIGS = [
    # name, instance, decoder, delta, tabu, iterations, B, |F|, phi_max, phi_steps, seed, every
    ("many_writers", lambda: synth.generate(20, 3, 8, 0.6, rs=0.25, seed=22), TIME, 6, 12, 25, 20, 3, 1, 3, 5, 1),
    ("phi0", lambda: synth.generate(30, 4, 10, 0.5, rs=0.3, seed=21), TIME, 8, 40, 30, 12, 4, 0, 5, 9, 1),
    ("fewer_searches", lambda: synth.generate(30, 4, 10, 0.5, rs=0.3, seed=31), TIME, 8, 20, 60, 3, 8, 1, 4, 2, 1),
    ("capacity", lambda: synth.generate(25, 4, 10, 0.6, rs=0.3, seed=33), CAP, 7, 16, 30, 6, 6, 2, 4, 7, 1),
    ("every3", lambda: synth.generate(25, 4, 10, 0.5, rs=0.3, seed=34), TIME, 7, 16, 31, 9, 3, 1, 3, 4, 3),
]
STATS = {}


@pytest.mark.parametrize("cfg", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_working_set_round_replay(cfg):
    name, make, dec, delta, tl, iters, B, NF, phi_max, phi_steps, seed, every = cfg
    orc = oracle.Oracle(make())
    o = orc.tabu_search(delta, tl, iters, searches=B, elite=NF, phi_max=phi_max, phi_steps=phi_steps, decoder=dec,
                        seed=seed, exchange_every=every, round_log=True)
    stats = STATS.setdefault(name, {})
    r = replay(orc, dec, delta, tl, iters, B, NF, phi_max, phi_steps, seed, every, stats)
    assert len(o["rounds"]) == len(r["rounds"]) == stats["rounds"]
    for i, (a, b) in enumerate(zip(o["rounds"], r["rounds"])):
        for key in ("C", "IC", "reads", "slot", "I_assigned", "C_read", "C_cur", "C_best"):
            assert a[key].tolist() == b[key], (name, i, key)
        assert a["W"].tolist() == b["W"], (name, i, "W")
    assert np.array_equal(o["trajectory"], r["trajectory"]), np.argwhere(o["trajectory"] != r["trajectory"])[:5]
    for key in ("best_makespan", "iterations_done", "evaluations", "elite_makespan"):
        assert o[key].tolist() == r[key], key
    assert o["best_order"].tolist() == r["best_order"]
    assert o["elite_order"].tolist() == r["elite_order"]


def test_replay_configs_cover_the_protocol():
    """The configurations above exercise every part of the round a plausible
    slip would touch: writes, writes refused because the record improved in
    the meantime, several writers of one record in a round, a best-since-read
    order that differs from the current one at the write, diversification
    that changes the makespan, exchanges forced by I_assigned running out,
    fewer searches than records and more."""
    for cfg in CONFIGS:
        if cfg[0] not in STATS:
            test_working_set_round_replay(cfg)
    tot = {k: sum(s[k] for s in STATS.values()) for k in next(iter(STATS.values()))}
    for k in ("writes", "rejected_writes", "multi_writer_rounds", "imp_differs_from_cur", "diversified",
              "diversify_changed_c", "expiry_fired"):
        assert tot[k] > 0, (k, tot)
    assert STATS["fewer_searches"]["expiry_fired"] > 0
    assert STATS["phi0"]["diversified"] > 0


def test_exchange_every_one_is_the_default():
    orc = oracle.Oracle(synth.generate(25, 4, 10, 0.5, rs=0.3, seed=34))
    kw = dict(searches=6, elite=3, phi_max=1, phi_steps=3, decoder=TIME, seed=4)
    a = orc.tabu_search(7, 16, 20, **kw)
    b = orc.tabu_search(7, 16, 20, exchange_every=1, **kw)
    c = orc.tabu_search(7, 16, 20, exchange_every=4, **kw)
    for k in ("trajectory", "best_makespan", "elite_order"):
        assert np.array_equal(a[k], b[k]), k
    assert not np.array_equal(a["trajectory"], c["trajectory"])
