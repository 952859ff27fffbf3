"""GPU parity on the benchmarked workloads at their stated lengths, and on
the search options of the C ABI that the other parity files do not cover
(rounds every k iterations, time budgets, the one-call batch entry point)."""
import hashlib
import os

import numpy as np
import pytest

import oracle
from paper_1711_04556_amd import synth
from tests.conftest import golden

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


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def _compare(g, o, elite=0):
    assert np.array_equal(g["trajectory"], o["trajectory"]), np.argwhere(g["trajectory"] != o["trajectory"])[:5]
    for k in ("best_makespan", "iterations_done", "evaluations", "best_order"):
        assert np.array_equal(g[k], o[k]), k
    if elite:
        assert np.array_equal(g["elite_makespan"], o["elite_makespan"])
        assert np.array_equal(g["elite_order"], o["elite_order"])


# ---------------------------------------------------------------------------
# The benchmarked workload: 480 cooperating searches x 1000 iterations on the
# 120-activity instance, compared with the oracle's full run (stored by
# tests/golden/make_plain480.py, which calls only the oracle).

@pytest.mark.parametrize("shape", ["registers", "lds"])
def test_headline_workload_full_length_equals_oracle(rc, shape):
    """Both launch shapes the benchmark's autotuner chooses between for this
    workload: the automatic one (256 threads, lane profiles in registers) and
    192 threads with 145-unit lane profiles in LDS and 8-bit finish times."""
    g0 = golden("plain480_ti.json")
    w = g0["workload"]
    inst = synth.instance_120_rs30(2)
    gi = rc.Instance(inst, eval=TIME)
    extra = dict(threads=192, profile_len=145) if shape == "lds" else {}
    plan = rc.SearchPlan(gi, rc.search_params(w["delta"], w["tabu_len"], w["iterations"], searches=w["searches"],
                                              elite=w["elite"], phi_max=w["phi_max"], phi_steps=w["phi_steps"],
                                              eval=TIME, seed=w["seed"], **extra))
    cfg = plan.config
    if shape == "lds":
        assert cfg["threads"] == 192 and cfg["finish_bits"] == 8 and cfg["lanes"] == 1
        assert cfg["register_profile"] == 0
    else:
        assert cfg["threads"] == 256 and cfg["register_profile"] == 1
    print(f"headline {shape}: {cfg}", flush=True)
    plan.run()
    g = plan.results()
    plan.close()
    assert g["best_makespan"].tolist() == g0["best_makespan"]
    assert g["iterations_done"].tolist() == g0["iterations_done"]
    assert [int(x) for x in g["evaluations"]] == g0["evaluations"]
    assert g["elite_makespan"].tolist() == g0["elite_makespan"]
    assert g["elite_order"].tolist() == g0["elite_order"]
    assert _digest(g["trajectory"]) == g0["trajectory_sha256"]
    assert _digest(g["best_order"]) == g0["best_order_sha256"]
    # the run is long enough for eq. 8's assignments to expire and for
    # diversified reads: the exchange pattern differs between searches
    assert len(set(g["best_makespan"].tolist())) > 1


@pytest.mark.parametrize("searches", [1, 4])
def test_fewer_searches_than_records(rc, searches):
    """B < |F| on the 120-activity instance: records that no search reads
    for a while, I_assigned running out (at most I_block / 5 = 60
    iterations per read) and reads cycling through all 16 records."""
    inst = synth.instance_120_rs30(2)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    kw = dict(searches=searches, elite=16, phi_max=3, phi_steps=20, seed=5)
    g = rc.tabu_search(gi, swap_range=20, tabu_len=329, iterations=300, **kw)
    o = orc.tabu_search(20, 329, 300, decoder=TIME, **kw)
    _compare(g, o, elite=16)


def test_batch_with_120_activity_members_at_192_threads(rc):
    """Batch members of 120 activities at the benchmark batch's dominant
    class shape (time-indexed, one candidate per lane, 192 threads, 8-bit
    finish times), beside smaller members, against the oracle."""
    # members 14, 20, 23 of the benchmark batch: 120 activities with
    # capacities below 128 (8-bit profile fields, one dword per time unit)
    batch = synth.mixed_batch(24, 3000)
    insts = [batch[k] for k in (0, 1, 14, 20, 23)]
    assert [i.n for i in insts] == [32, 62, 122, 122, 122] and all(max(i.capacity) < 128 for i in insts)
    gis, params = [], []
    for k, inst in enumerate(insts):
        d, tl = {32: (8, 60), 62: (14, 110), 122: (20, 329)}[inst.n]
        gis.append(rc.Instance(inst, eval=TIME))
        # 192 threads with a lane profile that fits (tight members of the
        # benchmark batch fall back to fewer threads with the automatic one)
        big = inst.n == 122
        params.append(rc.search_params(d, tl, 12, searches=32, elite=16, phi_max=3, phi_steps=20,
                                       threads=192 if big else 64, profile_len=140 if big else 0, seed=3000 + k))
    bt = rc.Batch(gis, params)
    info = bt.info
    assert 192 in info["class_threads"]
    bt.run()
    for k, inst in enumerate(insts):
        p = params[k]
        o = oracle.Oracle(inst).tabu_search(p.swap_range, p.tabu_len, p.iterations, searches=p.searches,
                                            elite=p.elite, phi_max=p.phi_max, phi_steps=p.phi_steps, decoder=TIME,
                                            seed=p.seed)
        _compare(bt.results(k), o, elite=16)
    bt.close()


# ---------------------------------------------------------------------------
# rounds every k iterations (Section 6.1 exchanges, exchange_every)

@pytest.mark.parametrize("dec,every", [(TIME, 3), (CAP, 5), (TIME, 40)])
def test_exchange_every_k_iterations(rc, dec, every):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=21)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=dec)
    kw = dict(searches=10, elite=4, phi_max=1, phi_steps=4, seed=9)
    plan = rc.SearchPlan(gi, rc.search_params(8, 40, 37, exchange_every=every, **kw))
    cfg = plan.config
    assert cfg["iteration_launches"] == -(-37 // every) and cfg["round_launches"] == 1 + (37 - 1) // every
    plan.run()
    g = plan.results()
    plan.close()
    o = orc.tabu_search(8, 40, 37, decoder=dec, exchange_every=every, **kw)
    _compare(g, o, elite=4)


def test_exchange_every_is_refused_where_rounds_are_per_iteration(rc):
    inst = synth.generate(20, 4, 10, 0.5, rs=0.3, seed=23)
    gi = rc.Instance(inst, eval=TIME)
    p = rc.search_params(6, 12, 5, searches=2, elite=2, exchange_every=2)
    with pytest.raises(rc.RcpspError) as e:
        rc.Batch([gi], [p])
    assert e.value.status == -1


# ---------------------------------------------------------------------------
# time budgets (reading: checked at iteration boundaries; eq. 8 keeps the
# allowance as I_block)

def test_time_budget_cooperative_run_is_a_shorter_run(rc):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=24)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=TIME)
    iters = 3000
    kw = dict(searches=12, elite=4, phi_max=2, phi_steps=4, seed=6)
    g = rc.tabu_search(gi, swap_range=8, tabu_len=40, iterations=iters, time_budget_us=3000, **kw)
    K = int(g["iterations_done"].max())
    print(f"budget run: {K} of {iters} iterations", flush=True)
    assert 1 <= K < iters
    o = orc.tabu_search(8, 40, K, decoder=TIME, i_block=iters, **kw)
    assert np.array_equal(g["trajectory"][:, :K], o["trajectory"])
    assert (g["trajectory"][:, K:] == -1).all()
    for k in ("best_makespan", "iterations_done", "evaluations", "best_order", "elite_makespan", "elite_order"):
        assert np.array_equal(g[k], o[k]), k


def test_time_budget_independent_searches_stop_on_their_own(rc):
    inst = synth.generate(30, 4, 10, 0.5, rs=0.3, seed=25)
    orc = oracle.Oracle(inst)
    gi = rc.Instance(inst, eval=CAP)
    iters = 4000
    g = rc.tabu_search(gi, swap_range=8, tabu_len=40, iterations=iters, searches=6, seed=3, time_budget_us=2000)
    done = g["iterations_done"]
    print(f"budget run: iterations per search {done.tolist()}", flush=True)
    assert done.min() >= 0 and done.max() < iters
    K = max(int(done.max()), 1)
    o = orc.tabu_search(8, 40, K, searches=6, decoder=CAP, seed=3)
    for b in range(6):
        kb = int(done[b])
        assert np.array_equal(g["trajectory"][b, :kb], o["trajectory"][b, :kb]), b
        assert (g["trajectory"][b, kb:] == -1).all()
        if kb:
            assert g["best_makespan"][b] == o["trajectory"][b, kb - 1, 3]
        assert orc.decode(g["best_order"][b], CAP) == g["best_makespan"][b]


def test_one_call_batch_entry_point(rc):
    insts = [synth.generate(n, 4, 10, 0.5, rs=0.3, seed=40 + n) for n in (20, 30, 45)]
    gis = [rc.Instance(i, eval=TIME) for i in insts]
    params = [rc.search_params(6, 20, 10, searches=5, elite=3 if k else 0, phi_max=2, phi_steps=3, seed=70 + k)
              for k in range(3)]
    outs = rc.tabu_search_batch(gis, params)
    for k, inst in enumerate(insts):
        p = params[k]
        o = oracle.Oracle(inst).tabu_search(6, 20, 10, searches=5, elite=p.elite, phi_max=2, phi_steps=3,
                                            decoder=TIME, seed=p.seed)
        _compare(outs[k], o, elite=p.elite)
