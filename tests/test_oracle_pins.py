"""Pins of the CPU oracle against what the paper prints and what the
mathematics fixes (worked examples, closed forms, invariants, brute force).

None of these tests re-uses oracle code to compute an expected value: the
expected values come from the paper's text, from hand derivations written in
the test, or from independent brute force in Python."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth
from tests.conftest import golden

TIME, CAP = oracle.TIME, oracle.CAPACITY


# --------------------------------------------------------------------------
# independent helpers (written from eqs. 2-4, not from the oracle)

def check_schedule(inst, start):
    """eq. 3 (precedence) and eq. 4 (per-time-unit capacity); returns C_max (eq. 2)."""
    N, M = inst.n, inst.m
    for i in range(N):
        for j in inst.succ[i]:
            assert start[j] >= start[i] + inst.duration[i], (i, j)
    cmax = max(start[i] + inst.duration[i] for i in range(N))
    for t in range(cmax + 1):
        for k in range(M):
            use = sum(inst.r(i, k) for i in range(N) if start[i] <= t < start[i] + inst.duration[i])
            assert use <= inst.capacity[k], (t, k, use)
    return cmax


def brute_force_optimum(inst):
    """Minimum makespan over all integer start-time vectors (eqs. 1-4)."""
    N, M = inst.n, inst.m
    real = list(range(1, N - 1))
    H = sum(inst.duration)
    grids = np.meshgrid(*[np.arange(0, H - inst.duration[i] + 1) for i in real], indexing="ij")
    S = np.stack([g.ravel() for g in grids], axis=1)  # [n_vec, n_real]
    ok = np.ones(len(S), dtype=bool)
    col = {a: c for c, a in enumerate(real)}
    for i in real:
        for j in inst.succ[i]:
            if j in col:
                ok &= S[:, col[j]] >= S[:, col[i]] + inst.duration[i]
    S = S[ok]
    d = np.array([inst.duration[i] for i in real])
    fin = S + d
    for t in range(H):
        active = (S <= t) & (t < fin)
        for k in range(M):
            rk = np.array([inst.r(i, k) for i in real])
            S_ok = (active * rk).sum(axis=1) <= inst.capacity[k]
            S, fin, active = S[S_ok], fin[S_ok], active[S_ok]
    return int(fin.max(axis=1).min()) if len(fin) else None


def all_feasible_orders(inst):
    N = inst.n
    pos_ok = []
    for perm in itertools.permutations(range(1, N - 1)):
        order = [0] + list(perm) + [N - 1]
        pos = {a: p for p, a in enumerate(order)}
        if all(pos[i] < pos[j] for i in range(N) for j in inst.succ[i]):
            pos_ok.append(order)
    return pos_ok


def table1():
    g = golden("table1.json")
    req = [x for pair in g["request"] for x in pair]
    return synth.Instance(n=12, m=2, duration=g["duration"], capacity=g["capacity"], request=req,
                          succ=g["successors"]), g


# --------------------------------------------------------------------------
# worked examples printed in the paper

def test_table1_critical_path_and_example_makespan():
    inst, g = table1()
    o = oracle.Oracle(inst)
    assert o.critical_path == g["critical_path"]
    W = g["example_order"]
    assert o.is_feasible_order(W)
    for dec in (TIME, CAP, 5):
        c, s = o.decode(W, dec, starts=True)
        assert c == g["example_makespan"]
        assert check_schedule(inst, s) == c


def test_table1_capacity_reading_is_unique():
    """Only capacities (6,6) reproduce the printed C_max = 22 among nearby readings."""
    inst, g = table1()
    hits = []
    for R0 in range(5, 9):
        for R1 in range(5, 9):
            i2 = synth.Instance(n=12, m=2, duration=inst.duration, capacity=[R0, R1], request=inst.request,
                                succ=inst.succ)
            if oracle.Oracle(i2).decode(g["example_order"], TIME) == g["example_makespan"]:
                hits.append((R0, R1))
    assert (6, 6) in hits


def test_fig5_capacity_update():
    g = golden("fig5_capacity_update.json")
    after, residual = oracle.capacity_update(g["capacity"], g["before"], g["request"], g["duration"], g["start"])
    assert after == g["after"]
    assert residual == 0


def test_table1_example_order_respects_levels():
    """The printed example order lists the levels of Section 4.1 one after another."""
    inst, g = table1()
    lv = oracle.Oracle(inst).levels()
    seq = [lv[a] for a in g["example_order"]]
    assert seq == sorted(seq)
    # levels by hand from the successor lists (unit-weight longest distance from 0)
    assert lv == [0, 1, 1, 2, 2, 3, 2, 3, 4, 4, 4, 5]


# --------------------------------------------------------------------------
# hand-derived cases

def test_time_vs_capacity_differ_hand_case():
    """N=5, one resource R=2; d=(0,5,1,3,0), r=(0,1,2,1,0), arcs 0->{1,2,3}->4,
    W=(0,1,2,3,4).  By hand: time-indexed puts 1 at [0,5), 2 at [5,6) and back-fills
    3 into [0,3) -> C_max 6; the capacity arrays after 1 and 2 are (5,0) then (6,6),
    so 3 starts at c[R-1] = 6 -> C_max 9."""
    inst = synth.Instance(n=5, m=1, duration=[0, 5, 1, 3, 0], capacity=[2], request=[0, 1, 2, 1, 0],
                          succ=[[1, 2, 3], [4], [4], [4], []])
    o = oracle.Oracle(inst)
    c_ti, s_ti = o.decode([0, 1, 2, 3, 4], TIME, starts=True)
    c_ci, s_ci = o.decode([0, 1, 2, 3, 4], CAP, starts=True)
    assert (c_ti, s_ti) == (6, [0, 0, 5, 0, 6])
    assert (c_ci, s_ci) == (9, [0, 0, 5, 6, 9])


def test_capacity_update_hand_case():
    """R=2, c=(0,0): r=1,d=5,s=0 gives (5,0); then r=2,d=1,s=5 gives (6,6)."""
    c, res = oracle.capacity_update(2, [0, 0], 1, 5, 0)
    assert (c, res) == ([5, 0], 0)
    c, res = oracle.capacity_update(2, c, 2, 1, 5)
    assert (c, res) == ([6, 6], 0)


# --------------------------------------------------------------------------
# closed forms

@pytest.mark.parametrize("seed", range(6))
def test_unlimited_capacity_gives_critical_path(seed):
    base = synth.generate(20, 3, 8, 0.7, rs=0.5, seed=100 + seed)
    cap = [sum(base.r(i, k) for i in range(base.n)) or 1 for k in range(base.m)]
    inst = synth.Instance(n=base.n, m=base.m, duration=base.duration, capacity=cap, request=base.request,
                          succ=base.succ)
    o = oracle.Oracle(inst)
    # longest path by hand: Bellman-style relaxation in id order (ids are topological)
    est = [0] * inst.n
    for i in range(inst.n):
        for j in inst.succ[i]:
            est[j] = max(est[j], est[i] + inst.duration[i])
    assert o.critical_path == est[-1]
    for t in range(5):
        W = synth.random_feasible_order(inst, seed * 10 + t)
        assert o.decode(W, TIME) == est[-1]
        assert o.decode(W, CAP) == est[-1]


@pytest.mark.parametrize("seed", range(4))
def test_full_capacity_requests_serialise(seed):
    """One resource, every real activity requests all R units: C_max = sum d."""
    base = synth.generate(12, 1, 6, 1.0, rs=0.5, seed=200 + seed)
    R = 5
    req = [0] + [R] * (base.n - 2) + [0]
    inst = synth.Instance(n=base.n, m=1, duration=base.duration, capacity=[R], request=req, succ=base.succ)
    o = oracle.Oracle(inst)
    for t in range(4):
        W = synth.random_feasible_order(inst, 50 + t)
        assert o.decode(W, TIME) == sum(inst.duration)
        assert o.decode(W, CAP) == sum(inst.duration)


def test_potential_move_count_closed_form():
    """|N_reduced| for u in [1,N-2], v in (u, min(u+delta, N-2)]."""
    for N, delta in [(12, 3), (32, 8), (122, 20), (302, 20), (10, 30)]:
        L = N - 2  # positions 1..N-2
        dd = min(delta, L - 1)
        closed = dd * L - dd * (dd + 1) // 2
        assert oracle.lib().orc_count_potential(N, delta) == closed


# --------------------------------------------------------------------------
# invariants on generated instances

@pytest.mark.parametrize("seed", range(8))
def test_decoders_produce_feasible_schedules(seed):
    inst = synth.generate(25, 4, 10, 0.5 + 0.05 * seed, rs=0.2 + 0.05 * seed, seed=300 + seed)
    o = oracle.Oracle(inst)
    for t in range(3):
        W = synth.random_feasible_order(inst, 7 * seed + t)
        for dec in (TIME, CAP):
            c, s = o.decode(W, dec, starts=True)
            assert check_schedule(inst, s) == c
            assert o.critical_path <= c <= o.horizon
            assert c == s[-1]


@pytest.mark.parametrize("seed", range(8))
def test_time_indexed_plain_equals_alg5(seed):
    inst = synth.generate(30, 4, 10, 0.6, rs=0.3, seed=400 + seed)
    o = oracle.Oracle(inst)
    for t in range(4):
        W = synth.random_feasible_order(inst, 11 * seed + t)
        assert o.decode(W, TIME, starts=True) == o.decode(W, 5, starts=True)


def test_capacity_update_invariants():
    """Alg. 4 keeps c non-increasing and places the whole effort when the
    activity was started at or after the eq. 7 earliest resource start."""
    rng = synth.Stream(99, 3)
    for trial in range(3000):
        R = 1 + rng.below(9)
        c = [0] * R
        for step in range(1 + rng.below(8)):
            r = 1 + rng.below(R)
            d = 1 + rng.below(5)
            s = c[R - r] + rng.below(4)
            c2, res = oracle.capacity_update(R, c, r, d, s)
            assert res == 0
            assert all(c2[i] >= c2[i + 1] for i in range(R - 1))
            c = c2


def _usage_envelope(acts, horizon):
    """Right envelope of the usage of one resource: at t, the largest total
    request of the placed activities at any time t' >= t."""
    use = [0] * (horizon + 1)
    for r, d, s in acts:
        for t in range(s, s + d):
            use[t] += r
    env = [0] * (horizon + 2)
    for t in range(horizon, -1, -1):
        env[t] = max(use[t], env[t + 1])
    return env


def test_capacity_update_never_optimistic():
    """Alg. 4 against the true right envelope of usage (the largest usage at
    or after t): the array c (unit j free from c[j] on) must never claim
    fewer busy units than the envelope at any t, so an activity started at
    eq. 7's time never overloads the resource.  It may claim more (it is
    conservative): the hand case R=2, (r=1,d=1,s=1) then (r=1,d=1,s=0)
    gives c=(2,1) while the envelope says one unit until 2 and none after."""
    c, _ = oracle.capacity_update(2, [0, 0], 1, 1, 1)
    c, _ = oracle.capacity_update(2, c, 1, 1, 0)
    assert c == [2, 1]
    assert _usage_envelope([(1, 1, 1), (1, 1, 0)], 3)[:3] == [1, 1, 0]
    rng = synth.Stream(123, 4)
    conservative = 0
    for trial in range(3000):
        R = 1 + rng.below(6)
        c = [0] * R
        acts = []
        for step in range(1 + rng.below(7)):
            r = 1 + rng.below(R)
            d = 1 + rng.below(4)
            s = c[R - r] + rng.below(3)      # at or after eq. 7's resource start
            c, res = oracle.capacity_update(R, c, r, d, s)
            assert res == 0
            acts.append((r, d, s))
            horizon = max(x[2] + x[1] for x in acts) + 1
            env = _usage_envelope(acts, horizon)
            busy = [sum(1 for cj in c if cj > t) for t in range(horizon + 1)]
            assert all(busy[t] >= env[t] for t in range(horizon + 1)), (R, acts, c)
            conservative += any(busy[t] > env[t] for t in range(horizon + 1))
    assert conservative > 0


# --------------------------------------------------------------------------
# brute force on tiny instances

TINY = [synth.random_tiny(s, n_real=4 + (s % 2), d_max=3 if s % 2 else 4) for s in range(40)]


@pytest.mark.parametrize("idx", range(len(TINY)))
def test_ssgs_min_over_orders_is_optimum(idx):
    inst = TINY[idx]
    o = oracle.Oracle(inst)
    opt = brute_force_optimum(inst)
    orders = all_feasible_orders(inst)
    ti = [o.decode(W, TIME) for W in orders]
    ci = [o.decode(W, CAP) for W in orders]
    assert min(ti) == opt
    # the capacity-indexed decoder never back-fills, yet some list still
    # reaches the optimum (an optimal schedule's activities by start time)
    assert min(ci) == opt
    for W in orders:
        for dec in (TIME, CAP):
            c, s = o.decode(W, dec, starts=True)
            assert check_schedule(inst, s) == c


@pytest.mark.parametrize("idx", range(0, len(TINY), 4))
def test_move_feasibility_equals_swap_then_check(idx):
    inst = TINY[idx]
    o = oracle.Oracle(inst)
    N = inst.n
    for W in all_feasible_orders(inst):
        for u in range(1, N - 1):
            for v in range(u + 1, N - 1):
                W2 = list(W)
                W2[u], W2[v] = W2[v], W2[u]
                pos = {a: p for p, a in enumerate(W2)}
                direct = all(pos[i] < pos[j] for i in range(N) for j in inst.succ[i])
                assert o.move_feasible(W, u, v) == direct


def test_evaluate_neighbourhood_against_direct_enumeration():
    inst = synth.generate(20, 3, 6, 0.6, rs=0.4, seed=555)
    o = oracle.Oracle(inst)
    N, delta = inst.n, 5
    rng = synth.Stream(5, 5)
    for t in range(4):
        W = synth.random_feasible_order(inst, t)
        tabu = np.zeros((N, N), np.uint8)
        for _ in range(15):
            u = 1 + rng.below(N - 3)
            tabu[u, min(u + 1 + rng.below(delta), N - 2)] = 1
        asp = o.decode(W, TIME) - 1
        mk, best = o.evaluate_neighbourhood(W, delta, TIME, tabu, asp)
        idx, cands = 0, []
        for u in range(1, N - 1):
            for v in range(u + 1, min(u + delta, N - 2) + 1):
                W2 = list(W)
                W2[u], W2[v] = W2[v], W2[u]
                pos = {a: p for p, a in enumerate(W2)}
                feas = all(pos[i] < pos[j] for i in range(N) for j in inst.succ[i])
                if feas:
                    c = o.decode(W2, TIME)
                    assert mk[idx] == c
                    cands.append((not (tabu[u, v] == 0 or c < asp), c, u, v))
                else:
                    assert mk[idx] == -1
                idx += 1
        assert idx == len(mk)
        cands.sort()
        assert best[:3] == [cands[0][2], cands[0][3], cands[0][1]]
        assert best[3] == len(cands)


# --------------------------------------------------------------------------
# Simple Tabu List and cache (Algs. 2, 3)

def test_stl_matches_last_added_moves():
    n, L = 20, 7
    ring_u = np.zeros(L, np.int32)
    ring_v = np.zeros(L, np.int32)
    widx = np.zeros(1, np.int32)
    cache = np.zeros(n * n, np.uint8)
    hist = []
    moves = [(u, v) for u in range(1, 18) for v in range(u + 1, min(u + 3, 18) + 1)]
    for step, mv in enumerate(moves[:40]):
        oracle.stl_add(ring_u, ring_v, widx, cache, n, *mv)
        hist.append(mv)
        recent = set(hist[-L:])
        for q in moves:
            assert oracle.stl_check(cache, n, *q) == (q in recent)
        assert widx[0] == (step + 1) % L


def test_stl_duplicate_eviction_is_literal():
    """Alg. 3 clears the cache bit when an older copy of a re-added move is
    evicted, even though a newer copy is still in the ring."""
    n, L = 10, 3
    ring_u, ring_v = np.zeros(L, np.int32), np.zeros(L, np.int32)
    widx, cache = np.zeros(1, np.int32), np.zeros(n * n, np.uint8)
    for mv in [(1, 2), (3, 4), (1, 2)]:
        oracle.stl_add(ring_u, ring_v, widx, cache, n, *mv)
    assert oracle.stl_check(cache, n, 1, 2)
    oracle.stl_add(ring_u, ring_v, widx, cache, n, 5, 6)   # evicts the first (1,2)
    assert not oracle.stl_check(cache, n, 1, 2)
    assert list(ring_u) == [5, 3, 1] and list(ring_v) == [6, 4, 2]


# --------------------------------------------------------------------------
# random numbers, initial orders, eq. 8

def test_splitmix64_known_answers():
    g = golden("splitmix64_seed0.json")
    gamma = 0x9E3779B97F4A7C15
    for k, hx in enumerate(g["outputs_hex"], start=1):
        assert oracle.mix64((k * gamma) & (2 ** 64 - 1)) == int(hx, 16)
        assert synth.mix64((k * gamma) & (2 ** 64 - 1)) == int(hx, 16)


def test_rng_counter_mode_definition():
    gamma, m = 0x9E3779B97F4A7C15, 2 ** 64 - 1
    for seed, stream, i in [(0, 0, 0), (1, 5, 7), (2 ** 63 + 5, 2 ** 32 + 3, 1000)]:
        key = synth.mix64((seed + (stream + 1) * gamma) & m)
        assert oracle.rng(seed, stream, i) == synth.mix64((key + (i + 1) * gamma) & m)


@pytest.mark.parametrize("seed", range(5))
def test_initial_orders_are_feasible_level_orders(seed):
    inst = synth.generate(60, 4, 10, 0.5, rs=0.4, seed=600 + seed)
    o = oracle.Oracle(inst)
    lv = o.levels()
    seen = set()
    for stream in range(6):
        W = o.initial_order(seed, stream)
        assert o.is_feasible_order(W)
        assert sorted(W) == list(range(inst.n))
        assert [lv[a] for a in W] == sorted(lv)
        seen.add(tuple(W))
    assert len(seen) > 1   # shuffling within levels gives different orders


def test_decay_table_tracks_exponential():
    import math
    E = oracle.decay_table()
    assert E[0] == 2 ** 24
    assert all(E[j] >= E[j + 1] for j in range(len(E) - 1))
    for j in range(0, 2000, 7):
        exact = 2 ** 24 * math.exp(-j / 256)
        assert abs(E[j] - exact) <= j + 1 + 1e-6 * exact


def test_iterations_assigned_closed_forms_and_bounds():
    for ib in (10, 100, 1000, 5000):
        # best record, untouched: quality 0.8 + intactness 0.2 -> the full quantity I_block / 5
        assert oracle.iterations_assigned(ib, 100, 100, 0) == ib // 5
        prev = None
        for ck in range(100, 140):
            ia = oracle.iterations_assigned(ib, ck, 100, 0)
            assert 1 <= ia <= max(1, ib // 5)
            if prev is not None:
                assert ia <= prev
            prev = ia
        prev = None
        for ic in range(0, 3 * ib, max(1, ib // 10)):
            ia = oracle.iterations_assigned(ib, 100, 100, ic)
            assert 1 <= ia <= max(1, ib // 5)
            if prev is not None:
                assert ia <= prev
            prev = ia
    # far from the best and long-used: quality -> 0, intactness -> 0.2 e^{-4 IC/I}
    import math
    ia = oracle.iterations_assigned(1000, 200, 100, 1000)
    assert ia == max(1, math.floor(1000 / 5 * 0.2 * math.exp(-4)))


# --------------------------------------------------------------------------
# tabu search self-consistency (the trajectory itself is parity-unpinned)

@pytest.mark.parametrize("dec", [TIME, CAP])
def test_single_search_replay_consistency(dec):
    inst = synth.single_instance_30(1)
    o = oracle.Oracle(inst)
    N, delta, TL, IT = inst.n, 8, 60, 60
    r = o.tabu_search(delta, TL, IT, searches=1, elite=0, decoder=dec, seed=1)
    W = o.initial_order(1, 0)
    best = o.decode(W, dec)
    ring_u, ring_v = np.zeros(TL, np.int32), np.zeros(TL, np.int32)
    widx, cache = np.zeros(1, np.int32), np.zeros(N * N, np.uint8)
    done = r["iterations_done"][0]
    for it in range(done):
        u, v, c, cb = r["trajectory"][0, it]
        mk, sel = o.evaluate_neighbourhood(W, delta, dec, cache.reshape(N, N), best)
        assert sel[:3] == [u, v, c]
        assert o.move_feasible(W, u, v)
        W[u], W[v] = W[v], W[u]
        assert o.decode(W, dec) == c
        oracle.stl_add(ring_u, ring_v, widx, cache, N, u, v)
        best = min(best, c)
        assert cb == best
    assert r["best_makespan"][0] == best
    assert o.decode(r["best_order"][0], dec) == best
    assert best >= o.critical_path
    traj = r["trajectory"][0, :done, 3]
    assert all(traj[i] >= traj[i + 1] for i in range(len(traj) - 1))
    assert r["evaluations"][0] > 0


def test_tabu_search_reaches_optimum_on_tiny_instances():
    hit = 0
    for inst in TINY[:20]:
        o = oracle.Oracle(inst)
        opt = brute_force_optimum(inst)
        r = o.tabu_search(3, 4, 40, searches=1, elite=0, decoder=TIME, seed=3)
        assert r["best_makespan"][0] >= opt
        hit += int(r["best_makespan"][0] == opt)
    assert hit >= 16


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_cooperative_search_invariants(dec):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=21)
    o = oracle.Oracle(inst)
    kw = dict(delta=8, tabu_len=40, iterations=40, searches=12, elite=4, phi_max=3, phi_steps=5,
              decoder=dec, seed=9)
    r1 = o.tabu_search(**kw)
    r2 = o.tabu_search(**kw)
    for k in r1:
        if r1[k] is not None:
            assert np.array_equal(r1[k], r2[k]), k
    cp = o.critical_path
    for b in range(12):
        assert r1["best_makespan"][b] == o.decode(r1["best_order"][b], dec)
        assert r1["best_makespan"][b] >= cp
        done = r1["iterations_done"][b]
        tr = r1["trajectory"][b, :done]
        # the best never rises, is never above the move just taken, and the
        # final best is the last row's
        assert (np.diff(tr[:, 3]) <= 0).all()
        assert (tr[:, 3] <= tr[:, 2]).all()
        assert done == 0 or tr[-1, 3] == r1["best_makespan"][b]
        assert (r1["trajectory"][b, done:] == -1).all()
    for k in range(4):
        assert r1["elite_makespan"][k] == o.decode(r1["elite_order"][k], dec)
        assert o.is_feasible_order(r1["elite_order"][k])


@pytest.mark.parametrize("dec", [oracle.TIME, oracle.CAPACITY])
def test_cut_short_search_is_prefix_of_full_allowance(dec):
    """A search stopped after K iterations (a time budget) while eq. 8 keeps
    the full allowance I_block = M: its trajectory is the first K rows of the
    search run for all M iterations, and i_block = iterations is the default."""
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=22)
    o = oracle.Oracle(inst)
    kw = dict(delta=8, tabu_len=40, searches=10, elite=4, phi_max=2, phi_steps=5, decoder=dec, seed=4)
    full = o.tabu_search(iterations=60, **kw)
    same = o.tabu_search(iterations=60, i_block=60, **kw)
    for k in full:
        if full[k] is not None:
            assert np.array_equal(full[k], same[k]), k
    differs = False
    for K in (1, 7, 23, 59):
        cut = o.tabu_search(iterations=K, i_block=60, **kw)
        assert np.array_equal(cut["trajectory"], full["trajectory"][:, :K])
        plain = o.tabu_search(iterations=K, **kw)
        differs = differs or not np.array_equal(plain["trajectory"], cut["trajectory"])
    # the allowance changes eq. 8's assignment, hence the exchange pattern
    assert differs
