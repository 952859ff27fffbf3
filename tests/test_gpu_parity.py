"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.  All results are integers and must match exactly."""
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


def _serial_instance():
    """One resource, every activity needs all of it: C_max = sum of durations,
    far beyond the default profile length (exercises the long-profile path)."""
    base = synth.generate(14, 1, 6, 1.0, rs=0.5, seed=77)
    req = [0] + [4] * (base.n - 2) + [0]
    return synth.Instance(n=base.n, m=1, duration=base.duration, capacity=[4], request=req, succ=base.succ,
                          name="serial14")


def _wide_instance():
    """Capacities above 127 force 16-bit profile fields (two dwords for M=4):
    a generated instance with every request and capacity tripled."""
    b = synth.generate(40, 4, 10, 0.75, rs=0.7, seed=3003)
    inst = synth.Instance(n=b.n, m=b.m, duration=b.duration, capacity=[3 * c for c in b.capacity],
                          request=[3 * r for r in b.request], succ=b.succ, name="wide40")
    assert max(inst.capacity) > 127
    return inst


EVAL_CASES = [
    ("table1", synth.table1_instance, 10),
    ("g30", lambda: synth.single_instance_30(1), 8),
    ("tiny", lambda: synth.random_tiny(5, n_real=5), 3),
    ("g60", lambda: synth.generate(60, 4, 10, 0.5, rs=0.4, seed=61), 14),
    ("wide40", _wide_instance, 12),
    ("m8", lambda: synth.generate(50, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=4001), 20),
    ("serial14", _serial_instance, 5),
    ("g120", synth.instance_120_rs30, 20),
    # capacity = the largest request: requests that take every unit
    ("rs0", lambda: synth.generate(40, 4, 10, 0.5, rs=0.0, seed=4014), 10),
    ("rs0m9rf1", lambda: synth.generate(36, 9, 10, 1.0, rs=0.0, seed=4015), 10),
]


@pytest.mark.parametrize("name,make,delta", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
@pytest.mark.parametrize("dec", [TIME, CAP])
def test_neighbourhood_parity(rc, name, make, delta, dec):
    inst = make()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    assert gi.info["eval"] == dec
    rng = synth.Stream(17, 3)
    for t in range(3):
        W = synth.random_feasible_order(inst, 100 + t) if t else orc.initial_order(5, 0)
        tabu = None
        asp = 2 ** 31 - 1
        if t == 2:
            tabu = np.zeros((inst.n, inst.n), np.uint8)
            for _ in range(3 * inst.n):
                u = 1 + rng.below(max(inst.n - 3, 1))
                v = min(u + 1 + rng.below(delta), inst.n - 2)
                if v > u:
                    tabu[u, v] = 1
            asp = orc.decode(W, dec)
        mk_g, best_g = gi.evaluate_neighbourhood(W, delta, tabu=tabu, aspiration=asp)
        mk_o, best_o = orc.evaluate_neighbourhood(W, delta, dec, tabu=tabu, aspiration=asp)
        assert np.array_equal(mk_g, mk_o), (name, t, np.nonzero(mk_g != mk_o)[0][:10])
        assert [best_g["u"], best_g["v"], best_g["makespan"], best_g["n_feasible"]] == best_o


def test_neighbourhood_edge_cases(rc):
    # one real activity: no potential move at all
    one = synth.Instance(n=3, m=1, duration=[0, 3, 0], capacity=[2], request=[0, 1, 0], succ=[[1], [2], []])
    gi = rc.Instance(one, eval=TIME)
    mk, best = gi.evaluate_neighbourhood([0, 1, 2], 4)
    assert mk.size == 0 and best == dict(u=0, v=0, makespan=-1, n_feasible=0)
    # a chain: every swap breaks a precedence arc
    chain = synth.Instance(n=6, m=1, duration=[0, 1, 2, 3, 4, 0], capacity=[1], request=[0, 1, 1, 1, 1, 0],
                           succ=[[1], [2], [3], [4], [5], []])
    gi = rc.Instance(chain, eval=CAP)
    mk, best = gi.evaluate_neighbourhood([0, 1, 2, 3, 4, 5], 3)
    assert (mk == -1).all() and best["n_feasible"] == 0
    # swap range beyond N
    inst = synth.single_instance_30(1)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    W = orc.initial_order(1, 3)
    mk_g, b_g = gi.evaluate_neighbourhood(W, 64)
    mk_o, b_o = orc.evaluate_neighbourhood(W, 64, TIME)
    assert np.array_equal(mk_g, mk_o)
    # an infeasible order is rejected
    bad = list(W)
    i = bad.index(inst.succ[0][0])
    bad[i], bad[-2] = bad[-2], bad[i]
    if not orc.is_feasible_order(bad):
        with pytest.raises(rc.RcpspError) as e:
            gi.evaluate_neighbourhood(bad, 8)
        assert e.value.status == -5


def test_neighbourhood_device_variant(rc):
    import torch
    inst = synth.generate(60, 4, 10, 0.5, rs=0.4, seed=62)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    W = orc.initial_order(2, 1)
    P = rc.potential_moves(inst.n, 14)
    order = torch.tensor(W, dtype=torch.int32, device="cuda")
    mk = torch.empty(P, dtype=torch.int32, device="cuda")
    best = torch.empty(4, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    gi.evaluate_neighbourhood_device(order, 14, mk, best, stream=s)
    torch.cuda.synchronize()
    mk_o, best_o = orc.evaluate_neighbourhood(W, 14, TIME)
    assert np.array_equal(mk.cpu().numpy(), mk_o)
    assert best.cpu().tolist() == best_o
    # invalid order: duplicate id -> n_feasible = RCPSP_E_ORDER, makespans untouched
    bad = list(W)
    bad[5] = bad[6]
    mk.fill_(7)
    gi.evaluate_neighbourhood_device(torch.tensor(bad, dtype=torch.int32, device="cuda"), 14, mk, best, stream=s)
    torch.cuda.synchronize()
    assert best.cpu().tolist()[3] == -5
    assert (mk.cpu().numpy() == 7).all()


def _compare_search(g, o, elite=0):
    assert np.array_equal(g["trajectory"], o["trajectory"]), np.argwhere(g["trajectory"] != o["trajectory"])[:5]
    assert np.array_equal(g["best_makespan"], o["best_makespan"])
    assert np.array_equal(g["iterations_done"], o["iterations_done"])
    assert np.array_equal(g["evaluations"], o["evaluations"])
    assert np.array_equal(g["best_order"], o["best_order"])
    if elite:
        assert np.array_equal(g["elite_makespan"], o["elite_makespan"])
        assert np.array_equal(g["elite_order"], o["elite_order"])


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_single_search_trajectory_30(rc, dec):
    """30 activities, 4 resources, one search, swap range 8, tabu list 60, 200 iterations, seed 1."""
    inst = synth.single_instance_30(1)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    kw = dict(swap_range=8, tabu_len=60, iterations=200, searches=1, elite=0, seed=1)
    g = rc.tabu_search(gi, **kw)
    o = orc.tabu_search(8, 60, 200, searches=1, elite=0, decoder=dec, seed=1)
    _compare_search(g, o)


@pytest.mark.parametrize("threads", [64, 128, 192, 256])
def test_independent_searches_any_launch_shape(rc, threads):
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=63)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    g = rc.tabu_search(gi, swap_range=14, tabu_len=110, iterations=40, searches=5, threads=threads, seed=4)
    o = orc.tabu_search(14, 110, 40, searches=5, decoder=TIME, seed=4)
    _compare_search(g, o)


@pytest.mark.parametrize("threads", [64, 192, 256])
def test_short_profile_overflow_path(rc, threads):
    """A 16-slot lane profile forces most candidates through the full-horizon
    re-decode (16-lane groups side by side); results must not change."""
    inst = synth.single_instance_30(1)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    g = rc.tabu_search(gi, swap_range=8, tabu_len=60, iterations=30, searches=2, profile_len=16, threads=threads,
                       seed=2)
    o = orc.tabu_search(8, 60, 30, searches=2, decoder=TIME, seed=2)
    _compare_search(g, o)
    assert g["overflow_decodes"] > 0


def test_overflow_redecode_counts_same_work(rc):
    """Candidates re-decoded after a lane-profile overflow count the same
    algorithmic operations as when the lane profile holds them."""
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=25)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=10, tabu_len=60, iterations=10, searches=4, seed=7, count_work=True, threads=192,
              full_decode=True)
    a = rc.tabu_search(gi, **kw)
    b = rc.tabu_search(gi, profile_len=16, **kw)
    for k in ("trajectory", "best_makespan", "evaluations"):
        assert np.array_equal(a[k], b[k]), k
    assert a["overflow_decodes"] == 0 and b["overflow_decodes"] > 0
    assert a["total_work"] == b["total_work"] > 0 and a["total_cells"] == b["total_cells"] > 0


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_cooperative_search_small(rc, dec):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=21)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    kw = dict(swap_range=8, tabu_len=40, iterations=40, searches=12, elite=4, phi_max=3, phi_steps=5, seed=9)
    g = rc.tabu_search(gi, **kw)
    o = orc.tabu_search(8, 40, 40, searches=12, elite=4, phi_max=3, phi_steps=5, decoder=dec, seed=9)
    _compare_search(g, o, elite=4)


def test_cooperative_search_many_exchanges(rc):
    """Short stints (I_block small) make searches exchange almost every
    iteration, including several writers and readers of one record per round."""
    inst = synth.generate(20, 3, 8, 0.6, rs=0.25, seed=22)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=6, tabu_len=12, iterations=25, searches=20, elite=3, phi_max=1, phi_steps=3, seed=5)
    g = rc.tabu_search(gi, **kw)
    o = orc.tabu_search(6, 12, 25, searches=20, elite=3, phi_max=1, phi_steps=3, decoder=TIME, seed=5)
    _compare_search(g, o, elite=3)


def test_plan_rerun_is_identical(rc):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=23)
    gi = rc.Instance(inst, eval=CAP)
    plan = rc.SearchPlan(gi, rc.search_params(8, 40, 30, searches=8, elite=4, phi_steps=5, seed=3))
    plan.run()
    a = plan.results()
    plan.run()
    b = plan.results()
    for k in ("trajectory", "best_makespan", "evaluations", "elite_order", "best_order"):
        assert np.array_equal(a[k], b[k]), k
    plan.close()


def test_plain_480_searches_full_size_short_run(rc):
    """The 120-activity workload (480 searches, working set 16, swap range 20,
    tabu list 329) in the launch configuration the benchmark times, for 3
    iterations: every trajectory record, best and working set match."""
    inst = synth.instance_120_rs30()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=20, tabu_len=329, iterations=3, searches=480, elite=16, phi_max=3, phi_steps=20, seed=2)
    g = rc.tabu_search(gi, **kw)
    o = orc.tabu_search(20, 329, 3, searches=480, elite=16, phi_max=3, phi_steps=20, decoder=TIME, seed=2)
    _compare_search(g, o, elite=16)


def test_plain_480_searches_full_run_properties(rc):
    """Full 1000-iteration run: properties that hold at any size, checked with
    the oracle's decoder on the returned orders."""
    inst = synth.instance_120_rs30()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst)
    dec = gi.info["eval"]
    g = rc.tabu_search(gi, swap_range=20, tabu_len=329, iterations=1000, searches=480, elite=16, phi_max=3,
                       phi_steps=20, seed=2)
    cp = orc.critical_path
    assert g["global_best"] >= cp
    assert g["global_best"] == min(g["best_makespan"].min(), g["elite_makespan"].min())
    for b in range(0, 480, 37):
        assert orc.is_feasible_order(g["best_order"][b])
        assert orc.decode(g["best_order"][b], dec) == g["best_makespan"][b]
        tr = g["trajectory"][b]
        done = g["iterations_done"][b]
        assert (tr[done:] == -1).all()
        assert (np.diff(tr[:done, 3]) <= 0).all()
    for k in range(16):
        assert orc.is_feasible_order(g["elite_order"][k])
        assert orc.decode(g["elite_order"][k], dec) == g["elite_makespan"][k]
    assert g["total_evaluations"] == g["evaluations"].sum() > 0


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_counting_and_timed_runs_match_graph_run(rc, dec):
    """The instrumented (work-counting) kernels and the event-timed eager run
    give the same search as the graph replay."""
    inst = synth.generate(40, 4, 10, 0.5, rs=0.3, seed=24)
    gi = rc.Instance(inst, eval=dec)
    kw = dict(swap_range=10, tabu_len=60, iterations=20, searches=10, elite=4, phi_steps=4, seed=6)
    plan = rc.SearchPlan(gi, rc.search_params(**kw))
    plan.run()
    a = plan.results()
    t = plan.run_timed()
    b = plan.results()
    assert t["iteration_ms"] > 0 and t["total_ms"] >= t["iteration_ms"]
    cplan = rc.SearchPlan(gi, rc.search_params(count_work=True, **kw))
    cplan.run()
    c = cplan.results()
    fplan = rc.SearchPlan(gi, rc.search_params(count_work=True, full_decode=True, **kw))
    fplan.run()
    f = fplan.results()
    for k in ("trajectory", "best_makespan", "evaluations", "elite_order", "best_order"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
        assert np.array_equal(a[k], f[k]), k
    # decoding every candidate from position 0 costs at least one operation
    # per activity; continuing from the shared prefix costs less, not nothing
    assert a["total_work"] == 0 and f["total_work"] > f["total_evaluations"] * inst.n
    assert 0 < c["total_work"] < f["total_work"]
    assert 0 < c["total_cells"] < c["total_work"] and 0 < f["total_cells"] < f["total_work"]
    plan.close()
    cplan.close()
    fplan.close()


def test_search_decoder_override(rc):
    """A search may use the other decoder than the instance's default."""
    inst = synth.generate(30, 4, 10, 0.5, rs=0.4, seed=25)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    g = rc.tabu_search(gi, swap_range=8, tabu_len=40, iterations=30, searches=4, elite=2, phi_steps=4,
                       eval=CAP, seed=8)
    o = orc.tabu_search(8, 40, 30, searches=4, elite=2, phi_steps=4, decoder=CAP, seed=8)
    _compare_search(g, o, elite=2)


def test_autotune_choice_is_a_valid_exact_plan(rc):
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=26)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst)
    base = rc.search_params(14, 110, 20, searches=32, elite=8, phi_steps=10, seed=3)
    tuned, info = rc.autotune(gi, base, trial_iterations=4)
    assert tuned.eval in (TIME, CAP) and tuned.threads in (64, 128, 256) and info["trials"] >= 2
    assert info["ns_per_evaluation"] > 0
    plan = rc.SearchPlan(gi, tuned)
    plan.run()
    g = plan.results()
    o = orc.tabu_search(14, 110, 20, searches=32, elite=8, phi_steps=10, decoder=tuned.eval, seed=3)
    _compare_search(g, o, elite=8)
    plan.close()


def _batch_case():
    insts, params = [], []
    for i, (n, rs, rf) in enumerate([(30, 0.5, 0.5), (60, 0.3, 0.75), (20, 0.7, 1.0), (40, 0.2, 0.25),
                                     (30, 0.6, 0.5), (50, 0.4, 0.5)]):
        insts.append(synth.generate(n, 4, 10, rf, rs=rs, seed=700 + i))
    insts.append(_wide_instance())
    return insts


def test_batch_matches_oracle_and_plans(rc):
    """Mixed sizes, decoders, iteration counts (0 and 1 included), threads,
    working-set and independent searches in one batch: every instance's
    results equal the oracle's and its own plan's."""
    insts = _batch_case()
    gis, params = [], []
    for i, inst in enumerate(insts):
        dec = TIME if i % 3 else CAP
        gis.append(rc.Instance(inst, eval=dec))
        elite = 0 if i % 4 == 1 else 4
        iters = [15, 9, 15, 1, 0, 15, 4][i]
        threads = [64, 64, 128, 64, 64, 128, 64][i]
        params.append(rc.search_params(6 + i % 3, 30, iters, searches=6 + i, elite=elite, phi_max=2, phi_steps=4,
                                       threads=threads, seed=11 + i))
    bt = rc.Batch(gis, params)
    info = bt.info
    assert info["instances"] == len(insts) and info["classes"] >= 2
    bt.run()
    for i, inst in enumerate(insts):
        g = bt.results(i)
        p = params[i]
        o = oracle.Oracle(inst).tabu_search(p.swap_range, p.tabu_len, p.iterations, searches=p.searches,
                                            elite=p.elite, phi_max=p.phi_max, phi_steps=p.phi_steps,
                                            decoder=gis[i].info["eval"], seed=p.seed)
        _compare_search(g, o, elite=p.elite)
        plan = rc.tabu_search(gis[i], swap_range=p.swap_range, tabu_len=p.tabu_len, iterations=p.iterations,
                              searches=p.searches, elite=p.elite, phi_max=p.phi_max, phi_steps=p.phi_steps,
                              threads=p.threads, seed=p.seed)
        _compare_search(g, plan, elite=p.elite)
    # a second run gives the same results
    first = [bt.results(i)["trajectory"] for i in range(len(insts))]
    bt.run()
    for i in range(len(insts)):
        assert np.array_equal(first[i], bt.results(i)["trajectory"])
    bt.close()


# ---------------------------------------------------------------------------
# Group decode: 16 lanes per candidate (time-indexed).  Same results as one
# candidate per lane and as the oracle.

GROUP_CASES = [
    ("g30", lambda: synth.single_instance_30(1), 8),
    ("g60", lambda: synth.generate(60, 4, 10, 0.5, rs=0.3, seed=63), 14),
    ("wide40", _wide_instance, 12),
    ("m8", lambda: synth.generate(50, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=4001), 20),
    ("serial14", _serial_instance, 5),
]


@pytest.mark.parametrize("name,make,delta", GROUP_CASES, ids=[c[0] for c in GROUP_CASES])
@pytest.mark.parametrize("threads", [64, 256])
def test_group_decode_search_parity(rc, name, make, delta, threads):
    inst = make()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=delta, tabu_len=30, iterations=25, searches=6, elite=3, phi_max=2, phi_steps=4, seed=8)
    plan = rc.SearchPlan(gi, rc.search_params(threads=threads, lanes=16, **kw))
    assert plan.config["lanes"] == 16
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(delta, 30, 25, searches=6, elite=3, phi_max=2, phi_steps=4, decoder=TIME, seed=8)
    _compare_search(g, o, elite=3)


def test_group_decode_overflow_path(rc):
    """A 16-unit profile per candidate sends most candidates through the
    group's long-profile decode; results must not change."""
    inst = synth.single_instance_30(1)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    g = rc.tabu_search(gi, swap_range=8, tabu_len=60, iterations=30, searches=2, profile_len=16, lanes=16, seed=2)
    o = orc.tabu_search(8, 60, 30, searches=2, decoder=TIME, seed=2)
    _compare_search(g, o)
    assert g["overflow_decodes"] > 0


def test_group_decode_counts_same_work(rc):
    """The instrumented group decode counts the same algorithmic operations
    as the one-lane decode (a property of the method, not of the launch)."""
    inst = synth.generate(40, 4, 10, 0.5, rs=0.3, seed=24)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=10, tabu_len=60, iterations=12, searches=6, elite=4, phi_steps=4, seed=6, count_work=True,
              full_decode=True)
    a = rc.tabu_search(gi, lanes=1, **kw)
    b = rc.tabu_search(gi, lanes=16, **kw)
    for k in ("trajectory", "best_makespan", "evaluations"):
        assert np.array_equal(a[k], b[k]), k
    assert a["total_work"] == b["total_work"] > 0


def test_large_instance_time_indexed_group(rc):
    """300 activities, 8 resources, durations 1..20: the per-lane profile does
    not fit; with 16 lanes per candidate and the time-indexed decoder the
    neighbourhood (the evaluation entry point's automatic layout) and a
    short cooperative search equal the oracle."""
    inst = synth.large_batch(1)[0]
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    W = orc.initial_order(3, 0)
    mk_g, best_g = gi.evaluate_neighbourhood(W, 20)
    mk_o, best_o = orc.evaluate_neighbourhood(W, 20, TIME)
    assert np.array_equal(mk_g, mk_o), np.nonzero(mk_g != mk_o)[0][:10]
    assert [best_g["u"], best_g["v"], best_g["makespan"], best_g["n_feasible"]] == best_o
    plan = rc.SearchPlan(gi, rc.search_params(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, seed=3,
                                              lanes=16))
    assert plan.config["lanes"] == 16 and plan.config["eval"] == TIME
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, decoder=TIME, seed=3)
    _compare_search(g, o, elite=4)


def test_batch_mixes_lane_and_group_decode(rc):
    insts = _batch_case()[:4]
    gis = [rc.Instance(i, eval=TIME) for i in insts]
    params = [rc.search_params(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4, threads=64,
                               lanes=(1 if k % 2 else 16), seed=40 + k) for k in range(len(insts))]
    bt = rc.Batch(gis, params)
    bt.run()
    for k, inst in enumerate(insts):
        o = oracle.Oracle(inst).tabu_search(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4, decoder=TIME,
                                            seed=40 + k)
        _compare_search(bt.results(k), o, elite=3)
    bt.close()


@pytest.mark.parametrize("threads,elite", [(64, 0), (192, 4)])
def test_lane_decode_after_requestless_activities(rc, threads, elite):
    """Most activities request no resource and last long: they never move a
    lane's resource frontier, so their successors start well past it, over
    units the lane has not written since an earlier candidate.  Every
    neighbourhood makespan and the whole search must equal the oracle."""
    for seed in (1301, 1302, 1303):
        inst = synth.generate(40, 4, 20, 0.2, rs=0.3, seed=seed)
        orc = oracle.Oracle(inst)
        gi = rc.Instance(inst, eval=TIME)
        for k in range(3):
            W = orc.initial_order(seed, k)
            mk_g, _ = gi.evaluate_neighbourhood(W, 12)
            mk_o, _ = orc.evaluate_neighbourhood(W, 12, TIME)
            assert np.array_equal(mk_g, mk_o), (seed, k, np.nonzero(mk_g != mk_o)[0][:10])
        kw = dict(swap_range=12, tabu_len=40, iterations=40, searches=8, elite=elite, phi_max=2, phi_steps=4,
                  seed=seed)
        g = rc.tabu_search(gi, threads=threads, **kw)
        o = orc.tabu_search(12, 40, 40, searches=8, elite=elite, phi_max=2, phi_steps=4, decoder=TIME, seed=seed)
        _compare_search(g, o, elite=elite)


# ---------------------------------------------------------------------------
# Capacity-indexed group decode: 8 lanes per candidate, a lane per resource.
# Same results as one candidate per lane and as the oracle.

CAP_GROUP_CASES = GROUP_CASES[:4] + [
    ("m12", lambda: synth.generate(40, 12, 10, 0.5, rs=0.5, seed=4012), 10),   # lanes own two resources
    ("m3", lambda: synth.generate(45, 3, 10, 0.7, rs=0.3, seed=4013), 12),     # lanes without a resource
    # capacity = the largest request (resource strength 0): updates whose
    # request takes every unit (Alg. 4 passes over nothing and raises all)
    ("rs0", lambda: synth.generate(40, 4, 10, 0.5, rs=0.0, seed=4014), 10),
    # every activity requests every resource, lanes own up to two
    ("rs0m9rf1", lambda: synth.generate(36, 9, 10, 1.0, rs=0.0, seed=4015), 10),
]


@pytest.mark.parametrize("name,make,delta", CAP_GROUP_CASES, ids=[c[0] for c in CAP_GROUP_CASES])
@pytest.mark.parametrize("threads", [64, 256, 512])
def test_capacity_group_decode_search_parity(rc, name, make, delta, threads):
    inst = make()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=CAP)
    kw = dict(swap_range=delta, tabu_len=30, iterations=25, searches=6, elite=3, phi_max=2, phi_steps=4, seed=8)
    plan = rc.SearchPlan(gi, rc.search_params(threads=threads, lanes=8, **kw))
    assert plan.config["lanes"] == 8 and plan.config["eval"] == CAP
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(delta, 30, 25, searches=6, elite=3, phi_max=2, phi_steps=4, decoder=CAP, seed=8)
    _compare_search(g, o, elite=3)


def test_capacity_group_decode_counts_same_work(rc):
    inst = synth.generate(40, 4, 10, 0.5, rs=0.3, seed=24)
    gi = rc.Instance(inst, eval=CAP)
    kw = dict(swap_range=10, tabu_len=60, iterations=12, searches=6, elite=4, phi_steps=4, seed=6, count_work=True,
              full_decode=True)
    a = rc.tabu_search(gi, lanes=1, **kw)
    b = rc.tabu_search(gi, lanes=8, **kw)
    for k in ("trajectory", "best_makespan", "evaluations"):
        assert np.array_equal(a[k], b[k]), k
    assert a["total_work"] == b["total_work"] > 0


def test_large_instance_capacity_group(rc):
    """300 activities, 8 resources: a short cooperative search with a lane
    per resource equals the oracle, independent searches too."""
    inst = synth.large_batch(1)[0]
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=CAP)
    plan = rc.SearchPlan(gi, rc.search_params(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, seed=3,
                                              lanes=8, threads=256))
    assert plan.config["lanes"] == 8 and plan.config["eval"] == CAP
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, decoder=CAP, seed=3)
    _compare_search(g, o, elite=4)
    g = rc.tabu_search(gi, swap_range=20, tabu_len=60, iterations=2, searches=3, seed=4, lanes=8, threads=128)
    o = orc.tabu_search(20, 60, 2, searches=3, decoder=CAP, seed=4)
    _compare_search(g, o)


def test_batch_mixes_capacity_lane_and_group_decode(rc):
    insts = _batch_case()[:4]
    gis = [rc.Instance(i, eval=CAP) for i in insts]
    params = [rc.search_params(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4, threads=64,
                               lanes=(1 if k % 2 else 8), seed=50 + k) for k in range(len(insts))]
    bt = rc.Batch(gis, params)
    bt.run()
    for k, inst in enumerate(insts):
        o = oracle.Oracle(inst).tabu_search(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4, decoder=CAP,
                                            seed=50 + k)
        _compare_search(bt.results(k), o, elite=3)
    bt.close()


def test_batch_autotune_groups_by_words_per_unit(rc):
    """Instances of one (N, M) whose capacities need 16-bit profile fields
    are tuned as a group of their own (they cannot take the 8-bit members'
    register profiles); the tuned batch equals the oracle for every member."""
    narrow = [synth.generate(30, 4, 10, 0.5, rs=0.4, seed=900 + k) for k in range(3)]
    wide = []
    for k in range(2):
        b = synth.generate(30, 4, 10, 0.75, rs=0.7, seed=910 + k)
        wide.append(synth.Instance(n=b.n, m=b.m, duration=b.duration, capacity=[3 * c for c in b.capacity],
                                   request=[3 * r for r in b.request], succ=b.succ, name=f"wide{k}"))
    insts = [narrow[0], wide[0], narrow[1], wide[1], narrow[2]]
    gis = [rc.Instance(i, eval=TIME) for i in insts]
    assert {g.info["field_bits"] for g in gis} == {8, 16}
    kw = dict(searches=4, elite=3, phi_max=2, phi_steps=4)
    params = [rc.search_params(7, 30, 8, eval=TIME, seed=70 + k, **kw) for k in range(len(insts))]
    tuned, info = rc.batch_autotune(gis, params, trial_iterations=2, sample=8)
    assert info["groups"] == 2
    assert sorted(info["group_members"][:2]) == [2, 3]
    bt = rc.Batch(gis, tuned)
    bt.run()
    for k, inst in enumerate(insts):
        o = oracle.Oracle(inst).tabu_search(7, 30, 8, decoder=TIME, seed=70 + k, **kw)
        _compare_search(bt.results(k), o, elite=3)
    bt.close()


@pytest.mark.parametrize("threads,profile_len,bits", [(192, 0, 8), (64, 300, 16), (128, 0, 8)])
def test_finish_time_width_and_three_waves(rc, threads, profile_len, bits):
    """Lane states hold 8-bit finish times while the lane profile is at most
    255 units and 16-bit beyond; 192 threads run three waves, each with its
    own base decode.  Same search as the oracle either way."""
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=64)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=12, tabu_len=60, iterations=30, searches=9, elite=4, phi_max=2, phi_steps=5, seed=12)
    plan = rc.SearchPlan(gi, rc.search_params(threads=threads, profile_len=profile_len, eval=TIME, **kw))
    cfg = plan.config
    assert cfg["threads"] == threads and cfg["finish_bits"] == bits and cfg["lanes"] == 1
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(12, 60, 30, searches=9, elite=4, phi_max=2, phi_steps=5, decoder=TIME, seed=12)
    _compare_search(g, o, elite=4)


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_host_driven_search_matches_homogeneous(rc, dec):
    """Heterogeneous model: the host runs the loop and the device evaluates
    each neighbourhood; trajectories equal the in-kernel search's and the
    oracle's, including a search that stops at the critical path."""
    for n, rs, seed, iters in ((40, 0.3, 66, 25), (20, 0.9, 67, 30)):
        inst = synth.generate(n, 4, 10, 0.5, rs=rs, seed=seed)
        gi = rc.Instance(inst, eval=dec)
        kw = dict(swap_range=10, tabu_len=40, iterations=iters, searches=3, seed=8)
        h = rc.tabu_search_hosted(gi, **kw)
        g = rc.tabu_search(gi, **kw)
        o = oracle.Oracle(inst).tabu_search(10, 40, iters, searches=3, decoder=dec, seed=8)
        _compare_search(h, o)
        _compare_search(g, o)
        assert h["global_best"] == g["global_best"] and h["total_evaluations"] == g["total_evaluations"]


def test_host_driven_search_arguments(rc):
    inst = synth.generate(20, 4, 10, 0.5, rs=0.3, seed=68)
    gi = rc.Instance(inst, eval=TIME)
    for bad in (dict(elite=2), dict(count_work=True), dict(eval=CAP)):
        with pytest.raises(rc.RcpspError) as e:
            rc.tabu_search_hosted(gi, **dict(dict(swap_range=6, tabu_len=20, iterations=5, searches=2, seed=1), **bad))
        assert e.value.status == -1


@pytest.mark.parametrize("dec", [TIME, CAP])
def test_forward_backward_improvement_of_initial_solutions(rc, dec):
    """Every second initial solution improved forward-backward before the
    search starts: independent searches and working-set records, against the
    oracle; the host-driven search takes the same initial orders."""
    inst = synth.generate(40, 4, 10, 0.5, rs=0.25, seed=69)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    kw = dict(swap_range=10, tabu_len=40, iterations=12, seed=4)
    g = rc.tabu_search(gi, searches=4, fbi=True, **kw)
    o = orc.tabu_search(10, 40, 12, searches=4, decoder=dec, seed=4, fbi=True)
    _compare_search(g, o)
    h = rc.tabu_search_hosted(gi, searches=4, fbi=True, **kw)
    _compare_search(h, o)
    g = rc.tabu_search(gi, searches=6, elite=4, phi_max=2, phi_steps=4, fbi=True, **kw)
    o = orc.tabu_search(10, 40, 12, searches=6, elite=4, phi_max=2, phi_steps=4, decoder=dec, seed=4, fbi=True)
    _compare_search(g, o, elite=4)
    # the improvement shortens at least one of these initial solutions
    assert any(orc.fbi(orc.initial_order(4, b), dec)[1] < orc.decode(orc.initial_order(4, b), dec) for b in (1, 3))


@pytest.mark.parametrize("dec,n", [(TIME, 800), (CAP, 300), (CAP, 800)])
def test_neighbourhood_large_instances(rc, dec, n):
    """Large instances (800 activities; capacity-indexed states that do not
    fit one per lane take 8 lanes per candidate): every makespan of the
    neighbourhood equals the oracle's.  At the activity limit (2,046 + 2
    dummies) the evaluation is either exact on sampled moves or refused with
    RCPSP_E_TOO_LARGE."""
    inst = synth.generate(n, 4, 10, 0.5, rs=0.5, seed=801)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    W = orc.initial_order(2, 0)
    mk_g, best_g = gi.evaluate_neighbourhood(W, 2)
    mk_o, best_o = orc.evaluate_neighbourhood(W, 2, dec)
    assert np.array_equal(mk_g, mk_o)
    assert [best_g["u"], best_g["v"], best_g["makespan"], best_g["n_feasible"]] == best_o
    for nb in (2046,):
        big = synth.generate(nb, 4, 10, 0.5, rs=0.5, seed=802)
        ob = oracle.Oracle(big)
        gb = rc.Instance(big, eval=dec)
        Wb = ob.initial_order(2, 0)
        try:
            mk_g, best_g = gb.evaluate_neighbourhood(Wb, 1)
        except rc.RcpspError as e:
            assert e.status == -9, e   # RCPSP_E_TOO_LARGE
            continue
        for j in range(0, len(mk_g), 97):
            u = 1 + j
            if mk_g[j] >= 0:
                w = list(Wb)
                w[u], w[u + 1] = w[u + 1], w[u]
                assert mk_g[j] == ob.decode(w, dec)


def _stretched(seed, factor):
    """Activities that request no resource made `factor` times longer: they
    never touch a lane's profile, so schedules run past 255 time units
    while every resource-requesting activity still fits a short profile."""
    b = synth.generate(40, 2, 20, 0.3, rs=0.2, seed=seed)
    d = list(b.duration)
    for i in range(1, b.n - 1):
        if all(b.r(i, k) == 0 for k in range(b.m)):
            d[i] *= factor
    return synth.Instance(n=b.n, m=b.m, duration=d, capacity=b.capacity, request=b.request, succ=b.succ,
                          name=f"stretched{seed}x{factor}")


def test_8bit_finish_times_past_255_hand_case(rc):
    """0->1->2->4, 0->3->4, one resource of 1 unit; d = (0, 250, 10, 1, 0),
    r = (0, 1, 0, 1, 0).  Order (0,1,3,2,4): 1 on [0,250), 3 on [250,251),
    2 (no request) on [250,260): C_max = 260, past what an 8-bit finish time
    holds.  By hand, the only feasible swap of (0,1,2,3,4) within range 2 is
    (2,3), giving 260; the order itself also gives 260."""
    inst = synth.Instance(n=5, m=1, duration=[0, 250, 10, 1, 0], capacity=[1], request=[0, 1, 0, 1, 0],
                          succ=[[1, 3], [2], [4], [4], []])
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    mk_g, best_g = gi.evaluate_neighbourhood([0, 1, 2, 3, 4], 2)
    assert mk_g.tolist() == [-1, -1, 260]
    assert [best_g["u"], best_g["v"], best_g["makespan"], best_g["n_feasible"]] == [2, 3, 260, 1]
    mk_o, best_o = orc.evaluate_neighbourhood([0, 1, 2, 3, 4], 2, TIME)
    assert mk_o.tolist() == mk_g.tolist()
    plan = rc.SearchPlan(gi, rc.search_params(2, 2, 6, searches=3, threads=64, seed=1))
    assert plan.config["finish_bits"] == 8
    plan.run()
    g = plan.results()
    plan.close()
    _compare_search(g, orc.tabu_search(2, 2, 6, searches=3, decoder=TIME, seed=1))


@pytest.mark.parametrize("seed,factor", [(1513, 3), (1508, 2), (1505, 2)])
@pytest.mark.parametrize("threads", [64, 192])
def test_8bit_finish_times_past_255(rc, seed, factor, threads):
    """Lane states with 8-bit finish times (profile at most 255 units) on
    instances whose schedules pass 255 through activities without requests:
    every such candidate must take the long-profile path, and neighbourhoods
    and searches equal the oracle."""
    inst = _stretched(seed, factor)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    past = 0
    for k in range(3):
        W = orc.initial_order(seed, k)
        mk_g, best_g = gi.evaluate_neighbourhood(W, 10)
        mk_o, best_o = orc.evaluate_neighbourhood(W, 10, TIME)
        assert np.array_equal(mk_g, mk_o), (k, np.nonzero(mk_g != mk_o)[0][:10])
        assert [best_g["u"], best_g["v"], best_g["makespan"], best_g["n_feasible"]] == best_o
        past += int((mk_o > 255).sum())
    assert past > 0
    for elite in (0, 4):
        kw = dict(swap_range=10, tabu_len=40, iterations=30, searches=6, elite=elite, phi_max=2, phi_steps=4,
                  seed=seed)
        # a lane profile of at most 255 units that fits the workgroup's LDS
        plan = rc.SearchPlan(gi, rc.search_params(threads=threads, eval=TIME, profile_len=200 if threads == 64
                                                  else 150, **kw))
        assert plan.config["finish_bits"] == 8 and plan.config["profile_len"] <= 255
        plan.run()
        g = plan.results()
        plan.close()
        o = orc.tabu_search(10, 40, 30, searches=6, elite=elite, phi_max=2, phi_steps=4, decoder=TIME, seed=seed)
        _compare_search(g, o, elite=elite)


# ---------------------------------------------------------------------------
# Register-resident lane profiles (160 time units of one dword per lane):
# same results as the LDS layouts and the oracle, including schedules that
# pass the register profile (long-profile path) or 255 (8-bit finish times).

REG_CASES = [
    ("table1", synth.table1_instance, 10),
    ("g30", lambda: synth.single_instance_30(1), 8),
    ("g60", lambda: synth.generate(60, 4, 10, 0.5, rs=0.3, seed=63), 14),
    ("g120", synth.instance_120_rs30, 20),
    ("serial14", _serial_instance, 5),
    ("stretched", lambda: _stretched(1513, 3), 10),
]


@pytest.mark.parametrize("name,make,delta", REG_CASES, ids=[c[0] for c in REG_CASES])
@pytest.mark.parametrize("elite", [0, 4])
def test_register_profile_search_parity(rc, name, make, delta, elite):
    inst = make()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=delta, tabu_len=30, iterations=25, searches=6, elite=elite, phi_max=2, phi_steps=4,
              seed=8)
    plan = rc.SearchPlan(gi, rc.search_params(lane_profile=2, eval=TIME, **kw))
    cfg = plan.config
    assert cfg["register_profile"] == 1 and cfg["threads"] == 256 and cfg["finish_bits"] == 8
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(delta, 30, 25, searches=6, elite=elite, phi_max=2, phi_steps=4, decoder=TIME, seed=8)
    _compare_search(g, o, elite=elite)
    if name == "stretched":
        assert g["overflow_decodes"] > 0   # schedules past the 160 register units


def test_register_profile_counts_same_work(rc):
    """The register decode counts the same algorithmic operations and cells
    as the LDS lane decode, from position 0 and with the shared prefix."""
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=24)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=10, tabu_len=60, iterations=12, searches=6, elite=4, phi_steps=4, seed=6, count_work=True,
              full_decode=True)
    a = rc.tabu_search(gi, lanes=1, threads=256, **kw)
    b = rc.tabu_search(gi, lane_profile=2, **kw)
    for k in ("trajectory", "best_makespan", "evaluations"):
        assert np.array_equal(a[k], b[k]), k
    assert a["total_work"] == b["total_work"] > 0 and a["total_cells"] == b["total_cells"] > 0


def test_register_profile_arguments(rc):
    gi = rc.Instance(_wide_instance(), eval=TIME)   # 16-bit fields, two dwords per unit: no register profile
    with pytest.raises(rc.RcpspError) as e:
        rc.SearchPlan(gi, rc.search_params(6, 20, 5, searches=2, lane_profile=2))
    assert e.value.status == -9
    gi = rc.Instance(synth.single_instance_30(1), eval=TIME)
    for bad in (dict(threads=64), dict(lanes=16)):
        with pytest.raises(rc.RcpspError) as e:
            rc.SearchPlan(gi, rc.search_params(6, 20, 5, searches=2, lane_profile=2, **bad))
        assert e.value.status == -1


# ---------------------------------------------------------------------------
# One candidate per wave (lanes = 64, 512 threads): the profile in the wave's
# registers, 2048 / words-per-unit time units per bank.  Same results as the
# oracle, including schedules past one bank (re-decoded over both) and past
# both (group decode over the full horizon).

def _scaled(make, k):
    """Every duration multiplied by k (makespans scale by k)."""
    def build():
        b = make()
        return synth.Instance(n=b.n, m=b.m, duration=[k * d for d in b.duration], capacity=b.capacity,
                              request=b.request, succ=b.succ, name=f"{b.name}x{k}")
    return build


def _m8_16bit():
    """8 resources with capacities above 127: four dwords per time unit
    (512 units per bank)."""
    b = synth.generate(50, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=4001)
    return synth.Instance(n=b.n, m=b.m, duration=b.duration, capacity=[3 * c for c in b.capacity],
                          request=[3 * r for r in b.request], succ=b.succ, name="m8x3")


WAVE_CASES = [
    ("table1", synth.table1_instance, 10, False),
    ("g30", lambda: synth.single_instance_30(1), 8, False),
    ("g60", lambda: synth.generate(60, 4, 10, 0.5, rs=0.3, seed=63), 14, False),
    ("wide40", _wide_instance, 12, False),
    ("m8", lambda: synth.generate(50, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=4001), 20, False),
    ("m8x3", _m8_16bit, 20, False),
    ("serial14", _serial_instance, 5, False),
    ("g30x33", _scaled(lambda: synth.single_instance_30(1), 33), 8, True),    # around one bank
    ("g30x66", _scaled(lambda: synth.single_instance_30(1), 66), 8, True),    # around both banks
    ("g30x80", _scaled(lambda: synth.single_instance_30(1), 80), 8, True),    # past both banks
]


@pytest.mark.parametrize("name,make,delta,long", WAVE_CASES, ids=[c[0] for c in WAVE_CASES])
@pytest.mark.parametrize("elite", [0, 4])
def test_wave_layout_search_parity(rc, name, make, delta, long, elite):
    inst = make()
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=delta, tabu_len=30, iterations=20, searches=6, elite=elite, phi_max=2, phi_steps=4,
              seed=8)
    plan = rc.SearchPlan(gi, rc.search_params(lanes=64, eval=TIME, **kw))
    cfg = plan.config
    assert cfg["lanes"] == 64 and cfg["threads"] == 512 and cfg["eval"] == TIME
    print(f"wave {name} elite {elite}: {cfg}", flush=True)
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(delta, 30, 20, searches=6, elite=elite, phi_max=2, phi_steps=4, decoder=TIME, seed=8)
    _compare_search(g, o, elite=elite)
    assert (g["overflow_decodes"] > 0) == long


def test_wave_layout_counts_same_work(rc):
    """Decoded from position 0 (every candidate over both banks after the
    loop), the wave decode counts the operations and cells of the lane
    decode; with the shared prefix it gives the same search."""
    inst = synth.generate(60, 4, 10, 0.5, rs=0.3, seed=24)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(swap_range=10, tabu_len=60, iterations=12, searches=6, elite=4, phi_steps=4, seed=6, count_work=True)
    a = rc.tabu_search(gi, lanes=1, threads=256, full_decode=True, **kw)
    b = rc.tabu_search(gi, lanes=64, full_decode=True, **kw)
    c = rc.tabu_search(gi, lanes=64, **kw)
    for k in ("trajectory", "best_makespan", "evaluations"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    assert a["total_work"] == b["total_work"] > 0 and a["total_cells"] == b["total_cells"] > 0
    assert 0 < c["total_work"] < b["total_work"]


def test_wave_layout_large_instance(rc):
    """300 activities, 8 resources, durations 1..20 (two dwords per unit,
    1024 units per bank): the automatic plan takes one candidate per wave;
    a cooperative search equals the oracle."""
    inst = synth.large_batch(1)[0]
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    plan = rc.SearchPlan(gi, rc.search_params(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, seed=3))
    assert plan.config["lanes"] == 64 and plan.config["eval"] == TIME
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(20, 60, 3, searches=4, elite=4, phi_max=2, phi_steps=4, decoder=TIME, seed=3)
    _compare_search(g, o, elite=4)


def test_batch_mixes_wave_lane_and_group_decode(rc):
    insts = _batch_case()[:4] + [_scaled(lambda: synth.single_instance_30(1), 33)()]
    gis = [rc.Instance(i, eval=TIME) for i in insts]
    lanes = [64, 1, 16, 64, 64]
    params = [rc.search_params(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4,
                               threads=512 if lanes[k] == 64 else 64, lanes=lanes[k], seed=40 + k)
              for k in range(len(insts))]
    bt = rc.Batch(gis, params)
    assert 512 in bt.info["class_threads"]
    bt.run()
    for k, inst in enumerate(insts):
        o = oracle.Oracle(inst).tabu_search(7, 30, 10, searches=5, elite=3, phi_max=2, phi_steps=4, decoder=TIME,
                                            seed=40 + k)
        _compare_search(bt.results(k), o, elite=3)
    bt.close()


def test_wave_layout_arguments(rc):
    gi = rc.Instance(synth.single_instance_30(1), eval=TIME)
    for bad in (dict(lanes=64, threads=256), dict(threads=512), dict(lanes=64, eval=CAP)):
        with pytest.raises(rc.RcpspError) as e:
            rc.SearchPlan(gi, rc.search_params(6, 20, 5, searches=2, **bad))
        assert e.value.status == -1, bad
