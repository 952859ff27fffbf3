"""Benchmark: SSGS neighbour evaluations per second of the tabu search on one
MI355X.

Headline (plain form): 480 seeded searches x 1000 iterations on one
120-activity instance (4 resources, resource strength 0.3, swap range 20,
tabu list 329, working set of 16 records, phi_max 3, phi_steps 20).  One step
= one whole search run from its initial state (every iteration of every
search plus the working-set exchange rounds), replayed from a captured HIP
graph; the instance and all search state are resident in HBM.

Batched leg: 1024 instances of 30/60/120 activities (resource factor and
strength varied), 32 searches each with a working set of 16, in one
persistent launch per class under a captured graph, against the plain form
(one plan per instance: a workgroup per search, a launch per iteration and
exchange round) on an evenly spaced sample of the same instances, with the
results of both compared.

Prints one JSON line on stdout (details on stderr)."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the serving leg runs one stream per launch class side by side; HIP maps
# streams onto this many hardware queues, and streams sharing a queue wait
# for each other's kernels (set before the HIP runtime starts)
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

METRIC = "SSGS neighbour evals/s (batched vs plain) at bit-exact makespan; p50/p99 latency"
PEAK_INT_OPS = 256 * 64 * 2.4e9      # 256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer op per lane-cycle
PEAK_LDS_BYTES = 256 * 128 * 2.4e9   # 256 CUs x 128 B per clock x 2.4 GHz
TRAFFIC_PROBE_BYTES = 1 << 30

WORKLOAD = dict(swap_range=20, tabu_len=329, iterations=1000, searches=480, elite=16, phi_max=3, phi_steps=20,
                seed=2)
# batched leg: swap range and tabu list by size (N incl. dummies); the tabu
# list is max(60, 0.15 x potential swaps), as for the plain workload
BATCH = dict(count=1024, base_seed=3000, searches=32, elite=16, phi_max=3, phi_steps=20, iterations=1000)
BATCH_DELTA_TL = {32: (8, 60), 62: (14, 110), 122: (20, 329)}
# serving leg: open-loop Poisson arrivals, 50 ms budget from admission
SERVE = dict(rate=2000.0, warmup_s=2.0, measure_s=10.0, budget_us=50000, searches=16, elite=16, iterations=1000,
             phi_max=3, phi_steps=20, seed=5, pool=256, max_active=1024, reduced_rate=500.0, reduced_measure_s=6.0)
SERVE_DELTA_TL = {32: (8, 60), 62: (14, 110), 122: (20, 329), 302: (20, 869)}
# large-instance leg: 256 instances of 300 activities, 8 resources; the
# workload's 2000 iterations take tens of minutes at the measured rate, so
# the first iterations are timed and the rate is reported
LARGE = dict(count=256, base_seed=4000, searches=16, elite=16, phi_max=3, phi_steps=20, iterations=16,
             swap_range=20, tabu_len=869)
# heterogeneous-model leg: independent searches of the plain workload's
# instance and move parameters, host-driven vs in-kernel
HOSTED = dict(searches=8, iterations=50)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_search_plain480_ti_hbm.txt")
TRAFFIC_SOURCES = ["paper_1711_04556_amd/csrc/rcpsp_device.h", "paper_1711_04556_amd/csrc/rcpsp_internal.h",
                   "paper_1711_04556_amd/csrc/rcpsp_host.cpp"]


def measured_traffic(cfg):
    """HBM bytes per iteration-kernel launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None when the library
    sources or the decoder differ from those the counters were taken on."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_SUMMARY):
            if ": " in line and not line.startswith((" ", "#", "|")):
                k, v = line.rstrip("\n").split(": ", 1)
                kv[k] = v
        h = hashlib.sha256()
        for f in TRAFFIC_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        # HBM bytes per launch come from the search state (orders, tabu lists,
        # records, the instance blob), which the decoder's profile length,
        # threads and lanes do not change; the decoder must match
        if kv.get("sources_sha256") != h.hexdigest() or kv.get("eval") != str(cfg["eval"]):
            return None
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def lds_bytes(work, cells, dec, nw, finish_bits):
    """Algorithmic LDS bytes of decodes from their counted work: every
    resource-state cell touched moves one packed profile unit (time-indexed:
    4 * dwords per unit, all resources of the unit) or one 16-bit capacity
    entry (capacity-indexed); every other operation (an activity placed, a
    predecessor finish time read) moves one finish time."""
    if dec == 1:
        return cells * 4 * nw + (work - cells) * (finish_bits // 8)
    return cells * 2 + (work - cells) * 2


SQ_SUMMARY = os.path.join(ROOT, "profiles", "k_search_plain480_ti_sq.txt")


def counter_fractions(cfg, avg_ms):
    """Counter-based fractions of the iteration kernel from the committed
    rocprofv3 SQ summary (per dispatch: SQ_INSTS_VALU, SQ_INSTS_LDS,
    SQ_WAVES, SQ_WAVE_CYCLES, SQ_WAIT_ANY), or None when the library sources
    or the launch shape differ from those the counters were taken on."""
    import hashlib
    try:
        kv = {}
        for line in open(SQ_SUMMARY):
            if ": " in line and not line.startswith((" ", "#", "|")):
                k, v = line.rstrip("\n").split(": ", 1)
                kv[k] = v
        h = hashlib.sha256()
        for f in TRAFFIC_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if kv.get("sources_sha256") != h.hexdigest():
            return None
        if any(kv.get(k) != str(cfg[k]) for k in ("eval", "threads", "profile_len", "lanes", "finish_bits")):
            return None
        valu, lds = float(kv["sq_insts_valu"]), float(kv["sq_insts_lds"])
        ms = float(kv["avg_launch_ms"])
        return {
            "source": os.path.relpath(SQ_SUMMARY, ROOT),
            "valu_lane_ops_per_s": valu * 64 / (ms * 1e-3),
            "valu_frac": valu * 64 / (ms * 1e-3) / PEAK_INT_OPS,
            "lds_bytes_per_s_at_4B_per_lane": lds * 256 / (ms * 1e-3),
            "lds_frac_at_4B_per_lane": lds * 256 / (ms * 1e-3) / PEAK_LDS_BYTES,
            "waves_per_launch": float(kv["sq_waves"]),
            "wait_share": float(kv["sq_wait_any"]) / float(kv["sq_wave_cycles"]),
            "valu_issue_share": float(kv["sq_insts_valu"]) / float(kv["sq_wave_cycles"]),
            "profiled_avg_launch_ms": ms,
            "bench_avg_launch_ms": avg_ms,
        }
    except (OSError, KeyError, ValueError, ZeroDivisionError):
        return None


def cpu_baseline(inst, decoder, iters=5):
    """The oracle (single thread, as it stands) on a bounded sample of the
    same workload: all 480 searches, the first `iters` iterations."""
    import oracle
    o = oracle.Oracle(inst)
    kw = dict(WORKLOAD)
    kw["iterations"] = iters
    t0 = time.perf_counter()
    r = o.tabu_search(kw["swap_range"], kw["tabu_len"], iters, searches=kw["searches"], elite=kw["elite"],
                      phi_max=kw["phi_max"], phi_steps=kw["phi_steps"], decoder=decoder, seed=kw["seed"],
                      trajectory=False)
    dt = time.perf_counter() - t0
    ev = int(r["evaluations"].sum())
    return dict(value=ev / dt, unit="evals/s", cores=1, kind="oracle",
                sample=f"480 searches x first {iters} iterations of the same workload "
                       f"({ev} evaluations in {dt:.1f} s, one host thread)")


def cpu_parallel(inst, decoder, passes=4):
    """The oracle's neighbourhood evaluation (as it stands) on the host's
    cores: the neighbourhoods of the workload's 480 initial orders, `passes`
    times, each thread taking whole orders (the paper's parallel CPU version
    splits one neighbourhood among threads; independent orders are the same
    decodes without synchronisation)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    o = oracle.Oracle(inst)
    orders = [o.initial_order(WORKLOAD["seed"], b) for b in range(WORKLOAD["searches"])]

    def evals(w):
        return o.evaluate_neighbourhood(w, WORKLOAD["swap_range"], decoder)[1][3]   # feasible moves decoded

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        ev = sum(ex.map(evals, orders * passes))
    dt = time.perf_counter() - t0
    return dict(value=ev / dt, unit="evals/s", cores=threads, kind="oracle",
                sample=f"neighbourhoods of the workload's 480 initial orders x {passes} ({ev} evaluations in "
                       f"{dt:.1f} s on {threads} threads)")


def batched_leg(rcpsp, synth, stream, steps, warmup, plain_sample=12):
    import torch
    t0 = time.perf_counter()
    insts = synth.mixed_batch(BATCH["count"], BATCH["base_seed"])
    gis = [rcpsp.Instance(i) for i in insts]
    params = []
    for k, inst in enumerate(insts):
        d, tl = BATCH_DELTA_TL[inst.n]
        params.append(rcpsp.search_params(d, tl, BATCH["iterations"], searches=BATCH["searches"],
                                          elite=BATCH["elite"], phi_max=BATCH["phi_max"],
                                          phi_steps=BATCH["phi_steps"], record_trajectory=False,
                                          seed=BATCH["base_seed"] + k))
    t1 = time.perf_counter()
    # trials on whole groups (up to 512 members): a 64-member sample has a
    # fifth of the tasks per iteration of its group, and there shapes that
    # hold a CU's whole LDS rank above shapes that run faster on the group
    params, tuning = rcpsp.batch_autotune(gis, params, trial_iterations=5, sample=512, stream=stream)
    tuning["seconds"] = time.perf_counter() - t1
    log("batch autotune", tuning)
    bt = rcpsp.Batch(gis, params, stream)
    info = bt.info
    log("batch", info, f"set-up {time.perf_counter() - t0:.1f} s")
    for _ in range(warmup):
        bt.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = [bt.results(k, stream, orders=False, trajectory=False) for k in range(len(insts))]
    evals = sum(r["total_evaluations"] for r in res)
    value = evals * steps / dt
    log(f"batched: {dt / steps * 1e3:.1f} ms/step, {evals} evaluations/step, {value:.4g} evals/s")
    # plain form on an evenly spaced sample: one plan per instance, run one after the other
    sample = list(range(0, len(insts), max(1, len(insts) // plain_sample)))[:plain_sample]
    p_ms = 0.0
    p_ev = 0
    exact = True
    s_work = s_cells = s_ev = 0
    for k in sample:
        q = type(params[k]).from_buffer_copy(params[k])
        q.threads = 0
        q.profile_len = 0
        plan = member_plan(rcpsp, gis[k], q, stream)
        plan.run(stream)
        timed = plan.run_timed(stream)
        r = plan.results(stream, orders=False, trajectory=False)
        plan.close()
        p_ms += timed["total_ms"]
        p_ev += r["total_evaluations"]
        exact = exact and r["total_evaluations"] == res[k]["total_evaluations"] and \
            r["global_best"] == res[k]["global_best"] and (r["best_makespan"] == res[k]["best_makespan"]).all()
        # the batch member's own shape, counting kernels: its algorithmic work
        c = type(params[k]).from_buffer_copy(params[k])
        c.count_work = 1
        cplan = member_plan(rcpsp, gis[k], c, stream)
        cplan.run(stream)
        cr = cplan.results(stream, orders=False, trajectory=False)
        cplan.close()
        s_work += cr["total_work"]
        s_cells += cr["total_cells"]
        s_ev += cr["total_evaluations"]
    plain = p_ev / (p_ms * 1e-3)
    sample_ev = sum(res[k]["total_evaluations"] for k in sample)
    log(f"plain sample: {len(sample)} instances, {p_ms:.1f} ms, {plain:.4g} evals/s, results equal: {exact}")
    ops_ev = s_work / max(s_ev, 1)
    achieved = value * ops_ev
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_INT_OPS / 1e12, unit="Tops/s",
                    frac=achieved / PEAK_INT_OPS, ops_per_evaluation=ops_ev,
                    basis=f"operations per evaluation counted on {len(sample)} sampled members in their own "
                          f"shape (instrumented kernels, {s_ev} evaluations) x the batch's evaluations per "
                          "second (all classes of the one graph)")
    cp = [g.info["critical_path"] for g in gis]
    dev = [100.0 * (r["global_best"] - c) / c for r, c in zip(res, cp)]
    return {
        "workload": f"{len(insts)} instances of 30/60/120 activities (4 resources, RF in .25..1, RS in .2..0.7), "
                    f"{BATCH['searches']} searches each, working set {BATCH['elite']}, {BATCH['iterations']} "
                    f"iterations, swap range 8/14/20, tabu list 60/110/329, phi_max 3, phi_steps 20",
        "value": value,
        "unit": "evals/s",
        "ms_per_step": dt / steps * 1e3,
        "steps": steps,
        "evaluations_per_step": evals,
        "roofline": roofline,
        "plain_value": plain,
        "plain_sample": f"{len(sample)} evenly spaced instances ({sample_ev} evaluations), one plan each, "
                        f"device time summed",
        "batched_vs_plain": value / plain,
        "results_equal_plain": bool(exact),
        "mean_cpm_dev_pct": sum(dev) / len(dev),
        "classes": info,
        "autotune": tuning,
    }


def hosted_leg(rcpsp, gi, dec, stream):
    """The same independent searches in the homogeneous model (the whole loop
    in one captured graph) and in the heterogeneous model (the host runs the
    loop, one device neighbourhood evaluation and read-back per iteration);
    wall time of each, results compared."""
    import numpy as np
    import torch
    kw = dict(WORKLOAD, searches=HOSTED["searches"], iterations=HOSTED["iterations"], elite=0, eval=dec)
    plan = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=True, **kw), stream)
    plan.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(stream)
    torch.cuda.synchronize()
    t_hom = time.perf_counter() - t0
    g = plan.results(stream)
    plan.close()
    rcpsp.tabu_search_hosted(gi, stream, **dict(kw, iterations=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = rcpsp.tabu_search_hosted(gi, stream, **kw)
    torch.cuda.synchronize()
    t_het = time.perf_counter() - t0
    equal = all(np.array_equal(g[k], h[k]) for k in ("trajectory", "best_makespan", "iterations_done",
                                                     "evaluations", "best_order"))
    its = int(np.asarray(h["iterations_done"]).sum())
    out = dict(workload=f"{HOSTED['searches']} independent searches x {HOSTED['iterations']} iterations on the "
                        "plain workload's instance (swap range 20, tabu list 329)",
               homogeneous_ms=1e3 * t_hom, hosted_ms=1e3 * t_het, search_iterations=its,
               hosted_us_per_iteration=1e6 * t_het / max(its, 1),
               homogeneous_evals_per_s=h["total_evaluations"] / t_hom,
               hosted_evals_per_s=h["total_evaluations"] / t_het,
               homogeneous_speedup=t_het / t_hom, results_equal=bool(equal))
    log("hosted", out)
    return out


def convergence_leg(rcpsp, gi, dec, stream, seeds, searches=(1, 4, 16, 64, 256, 480)):
    """Best makespan against iterations for different numbers of cooperating
    searches (working set 16) on the plain workload's instance, each point the
    mean over `seeds` seeded runs of 1000 iterations; 480 independent
    searches (no working set) as the reference without cooperation.  The
    best after iteration i is the global best: the minimum over the searches
    of their best after i + 1 iterations and over the working set's records.
    A record only ever receives a search's best since its read (never below
    that search's best), so the records' part is their initial makespans
    (those no search has read when there are fewer searches than records),
    read from a run of no iteration."""
    import numpy as np
    checkpoints = (0, 9, 49, 99, 249, 499, 999)
    rows = []
    t0 = time.perf_counter()
    for B, elite in [(b, 16) for b in searches] + [(480, 0)]:
        curves = []
        for k in range(seeds):
            kw = dict(WORKLOAD, searches=B, elite=elite, eval=dec, seed=1000 + k)
            plan = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=True, **kw), stream)
            plan.run(stream)
            r = plan.results(stream, orders=False)
            plan.close()
            rec0 = np.iinfo(np.int32).max
            if elite:
                p0 = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=False, **dict(kw, iterations=0)),
                                      stream)
                p0.run(stream)
                rec0 = int(p0.results(stream, orders=False, trajectory=False)["elite_makespan"].min())
                p0.close()
            traj = np.asarray(r["trajectory"])[:, :, 3].astype(np.int64)   # best per search per iteration
            # iterations not run (a search stopped early) keep the last best
            best = np.where(traj < 0, np.iinfo(np.int32).max, traj)
            best = np.minimum(np.minimum.accumulate(best, axis=1).min(axis=0), rec0)
            curves.append(best)
        c = np.mean(np.asarray(curves, dtype=np.float64), axis=0)
        rows.append(dict(searches=B, working_set=elite,
                         mean_best={str(i + 1): round(float(c[i]), 2) for i in checkpoints}))
        log("convergence", rows[-1], f"{time.perf_counter() - t0:.0f} s")
    return dict(workload="plain workload's instance, 1000 iterations, cooperative searches with working set 16 "
                         f"and 480 independent searches; mean over {seeds} seeds (1000..{999 + seeds})",
                rows=rows)


def reselect_leg(rcpsp, gi, stream, period, probe, threads, profile_len, periods=2):
    """Periodic decoder re-selection on the plain workload (480 searches,
    working set 16), `periods` periods of `period` iterations, each starting
    with `probe` timed iterations of both decoders: wall time against the
    same iterations with each decoder fixed, and the segment log.  threads
    and profile_len shape the time-indexed decoder (the capacity-indexed one
    takes its automatic shape)."""
    import torch
    iters = period * periods
    kw = dict(WORKLOAD, iterations=iters, record_trajectory=False, threads=threads, profile_len=profile_len)
    t = {}
    for name, dec in (("time", 1), ("capacity", 2)):
        shape = {} if dec == 1 else dict(threads=0, profile_len=0)
        plan = rcpsp.SearchPlan(gi, rcpsp.search_params(**dict(kw, eval=dec, **shape)), stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(stream)
        torch.cuda.synchronize()
        t[name] = time.perf_counter() - t0
        r = plan.results(stream, orders=False)
        t[name + "_best"] = r["global_best"]
        plan.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, segs = rcpsp.tabu_search_reselect(gi, period, probe, stream, **kw)
    torch.cuda.synchronize()
    t_rs = time.perf_counter() - t0
    out = dict(workload=f"plain workload, {iters} iterations, period {period}, probe {probe}",
               reselect_ms=1e3 * t_rs, time_fixed_ms=1e3 * t["time"], capacity_fixed_ms=1e3 * t["capacity"],
               best=dict(reselect=r["global_best"], time=t["time_best"], capacity=t["capacity_best"]),
               segments=[dict(first=s["first_iteration"], n=s["iterations"], eval=s["eval"], probe=s["probe"],
                              ms_per_iteration=round(s["ms_per_iteration"], 4)) for s in segs])
    log("reselect", out)
    return out


def large_leg(rcpsp, synth, stream, steps):
    import torch
    t0 = time.perf_counter()
    insts = synth.large_batch(LARGE["count"], LARGE["base_seed"])
    gis = [rcpsp.Instance(i) for i in insts]
    base = rcpsp.search_params(LARGE["swap_range"], LARGE["tabu_len"], LARGE["iterations"],
                               searches=LARGE["searches"], elite=LARGE["elite"], phi_max=LARGE["phi_max"],
                               phi_steps=LARGE["phi_steps"], record_trajectory=False, seed=LARGE["base_seed"])
    t1 = time.perf_counter()
    params, tuning = rcpsp.batch_autotune(gis, base, trial_iterations=1, sample=16, stream=stream)
    tuning["seconds"] = time.perf_counter() - t1
    log("large autotune", tuning)
    bt = rcpsp.Batch(gis, params, stream)
    info = bt.info
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = [bt.results(k, stream, orders=False, trajectory=False) for k in range(len(insts))]
    evals = sum(r["total_evaluations"] for r in res)
    bt.close()
    # algorithmic work per evaluation: two members as plans of their own
    # shape with the counting kernels (same searches, same evaluations)
    s_work = s_cells = s_ev = 0
    for k in (0, len(insts) // 2):
        c = type(params[k]).from_buffer_copy(params[k])
        c.count_work = 1
        cplan = member_plan(rcpsp, gis[k], c, stream)
        cplan.run(stream)
        cr = cplan.results(stream, orders=False, trajectory=False)
        cplan.close()
        assert cr["total_evaluations"] == res[k]["total_evaluations"]
        s_work += cr["total_work"]
        s_cells += cr["total_cells"]
        s_ev += cr["total_evaluations"]
    value = evals * steps / dt
    ops_ev = s_work / max(s_ev, 1)
    cpm = [100.0 * (r["global_best"] - g.info["critical_path"]) / g.info["critical_path"] for r, g in zip(res, gis)]
    out = {
        "workload": f"{len(insts)} instances of 300 activities (8 resources, durations 1..20, capacities 10..60), "
                    f"{LARGE['searches']} searches and working set {LARGE['elite']} each, swap range 20, tabu list "
                    f"869, {LARGE['iterations']} iterations timed (the workload's 2000 would take "
                    f"{dt / steps / LARGE['iterations'] * 2000 / 60:.0f} min at this rate)",
        "value": value,
        "unit": "evals/s",
        "iterations_timed": LARGE["iterations"],
        "ms_per_iteration": dt / steps / LARGE["iterations"] * 1e3,
        "evaluations_per_step": evals,
        "mean_cpm_dev_pct": sum(cpm) / len(cpm),
        "roofline": dict(bound="alu", achieved=value * ops_ev / 1e12, peak=PEAK_INT_OPS / 1e12, unit="Tops/s",
                         frac=value * ops_ev / PEAK_INT_OPS, ops_per_evaluation=ops_ev,
                         cells_per_evaluation=s_cells / max(s_ev, 1),
                         basis="operations per evaluation counted on two members run as plans of their own shape "
                               "(instrumented kernels) x the batch's evaluations per second"),
        "classes": info,
        "autotune": tuning,
    }
    log("large", out)
    return out


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def serving_leg(rcpsp, synth, stream, rate, warmup_s, measure_s, big_threads=128):
    """Config: Poisson arrivals at `rate`/s, sizes uniform over 30/60/120/300
    activities, 16 searches and a working set of 16 per request, 50 ms
    budget from admission.  Latency = time the result is available to the
    caller minus the scheduled arrival."""
    import numpy as np
    t0 = time.perf_counter()
    pool = synth.serving_pool(SERVE["pool"])
    gis = {n: [rcpsp.Instance(i) for i in lst] for n, lst in pool.items()}
    params = {}
    tuning = {}
    for n, lst in gis.items():
        d, tl = SERVE_DELTA_TL[n + 2]
        big = n >= 300
        base = rcpsp.search_params(d, tl, SERVE["iterations"], searches=SERVE["searches"], elite=SERVE["elite"],
                                   phi_max=SERVE["phi_max"], phi_steps=SERVE["phi_steps"],
                                   threads=big_threads if big else 64, lanes=8 if big else 0,
                                   eval=rcpsp.EVAL_CAPACITY if big else rcpsp.EVAL_AUTO,
                                   record_trajectory=False, seed=SERVE["seed"])
        # decoder and lanes per size from the batch autotuner on a sample, at
        # one wave per search for the sizes that share the time-indexed launch
        # class (classes split the CUs between them).  The 300-activity size
        # is a class of its own with the longest tasks; the autotuner ranks
        # shapes by one iteration's throughput, which says nothing about task
        # length, so it takes the shape measured best for serving latency:
        # capacity-indexed, 8 lanes per candidate, 512 threads (one search
        # per CU: an iteration of a request's 16 searches in ~0.1 s, where
        # 128 threads took longer than the budget)
        tuned, info = rcpsp.batch_autotune(lst[:8], base, trial_iterations=1, sample=8, stream=stream)
        params[n] = tuned[0]
        tuning[str(n)] = dict(eval=info["group_eval"][0], threads=info["group_threads"][0],
                              lanes=info["group_lanes"][0])
    log("serving set-up", f"{time.perf_counter() - t0:.1f} s", tuning)
    arrivals = synth.serving_arrivals(rate, warmup_s + measure_s, SERVE["seed"])
    sizes = synth.SERVING_SIZES
    srv = rcpsp.Server(max_active=SERVE["max_active"], slice_us=1000, arena_bytes=8 << 30)
    counters = {n: 0 for n in sizes}
    info_of = {}
    start = srv.now_ns() + 50_000_000
    j = 0
    recs = []
    deadline = start + int((warmup_s + measure_s + 30.0) * 1e9)
    next_log = start + 1_000_000_000
    while (j < len(arrivals) or info_of) and srv.now_ns() < deadline:
        now = srv.now_ns()
        if now >= next_log:
            next_log += 1_000_000_000
            log(f"serving t={(now - start) * 1e-9:.0f} s: submitted {j}, finished {len(recs)}, "
                f"in flight {len(info_of)}")
        while j < len(arrivals) and start + int(arrivals[j][0] * 1e9) <= now:
            n = sizes[arrivals[j][1]]
            k = counters[n]
            counters[n] += 1
            p = type(params[n]).from_buffer_copy(params[n])
            p.seed = SERVE["seed"] + j
            t = srv.submit(gis[n][k % len(gis[n])], p, SERVE["budget_us"])
            info_of[t] = (j, n, start + int(arrivals[j][0] * 1e9))
            j += 1
        done = srv.take_finished()
        for t in done:
            st = srv.poll(t)
            jj, n, sched = info_of.pop(t)
            recs.append((jj, n, sched, st))
            srv.release(t)
        if not done:
            nxt = start + int(arrivals[j][0] * 1e9) if j < len(arrivals) else now + 200_000
            wait = min(nxt - srv.now_ns(), 200_000)
            if wait > 50_000:
                time.sleep(wait * 1e-9 * 0.5)
    unfinished = len(info_of)
    stats = srv.stats
    srv.close()
    lo, hi = start + int(warmup_s * 1e9), start + int((warmup_s + measure_s) * 1e9)
    meas = [r for r in recs if lo <= r[2] < hi]
    ok = [r for r in meas if r[3]["state"] == rcpsp.REQ_DONE]
    lat = [(r[3]["seen_ns"] - r[2]) * 1e-6 for r in ok]
    lat_dev = [(r[3]["done_ns"] - r[2]) * 1e-6 for r in ok]
    queue = [(r[3]["admit_ns"] - r[2]) * 1e-6 for r in ok]
    submit_lag = [(r[3]["submit_ns"] - r[2]) * 1e-6 for r in ok]
    admit_wait = [(r[3]["admit_ns"] - r[3]["submit_ns"]) * 1e-6 for r in ok]
    run_time = [(r[3]["done_ns"] - r[3]["admit_ns"]) * 1e-6 for r in ok]
    evals = sum(r[3]["evaluations"] for r in ok)
    per_size = {}
    for n in sizes:
        rs = [r for r in ok if r[1] == n]
        if rs:
            per_size[str(n)] = dict(requests=len(rs), p50_ms=pct([(r[3]["seen_ns"] - r[2]) * 1e-6 for r in rs], 50),
                                    p99_ms=pct([(r[3]["seen_ns"] - r[2]) * 1e-6 for r in rs], 99),
                                    iterations_p50=pct([r[3]["iterations"] for r in rs], 50),
                                    evals_per_request=sum(r[3]["evaluations"] for r in rs) / len(rs))
    out = {
        "workload": f"open-loop Poisson arrivals at {rate:g}/s for {warmup_s + measure_s:g} s "
                    f"({len(arrivals)} requests; latency over the {measure_s:g} s after a {warmup_s:g} s "
                    f"warm-up), sizes uniform over 30/60/120/300 activities ({SERVE['pool']} distinct instances "
                    f"per size, cycled), {SERVE['searches']} searches and working set {SERVE['elite']} per "
                    f"request, {SERVE['budget_us'] // 1000} ms budget from admission, allowance "
                    f"{SERVE['iterations']} iterations, at most {SERVE['max_active']} requests resident",
        "requests_measured": len(meas),
        "completed": len(ok),
        "unfinished_at_cutoff": unfinished,
        "p50_ms": pct(lat, 50),
        "p99_ms": pct(lat, 99),
        "p50_ms_device_end": pct(lat_dev, 50),
        "p99_ms_device_end": pct(lat_dev, 99),
        "queueing_p99_ms": pct(queue, 99),
        "submit_lag_p50_ms": pct(submit_lag, 50),
        "admission_wait_p50_ms": pct(admit_wait, 50),
        "admission_wait_p99_ms": pct(admit_wait, 99),
        "admitted_to_end_p50_ms": pct(run_time, 50),
        "admitted_to_end_p99_ms": pct(run_time, 99),
        "evals_per_s": evals / measure_s,
        "per_size": per_size,
        "tuning": tuning,
        "device_clock_mhz": stats["device_clock_mhz"],
        "slices": stats["slices"],
        "slice_busy_ms_mean": stats["busy_ms"] / max(stats["slices"], 1),
    }
    log("serving", out)
    return out


def lds_words(info):
    """Dwords per packed time unit of the time-indexed profile (8-bit fields:
    four resources per dword; 16-bit: two)."""
    per = 4 if info["field_bits"] == 8 else 2
    return max(1, -(-info["m"] // per))


def member_plan(rcpsp, gi, q, stream):
    """A plan of a batch member's parameters, with the fallbacks the batch
    itself takes when a member's workgroup does not fit: the lane profile
    in LDS instead of registers, then fewer threads."""
    q = type(q).from_buffer_copy(q)
    while True:
        try:
            return rcpsp.SearchPlan(gi, q, stream)
        except rcpsp.RcpspError as e:
            if e.status != -9:
                raise
            if q.lane_profile == 2:
                q.lane_profile = 1
            elif q.threads > 64:
                q.threads = 128 if q.threads == 192 else q.threads // 2
            else:
                raise


def count_work(rcpsp, gi, kw, stream, evals, full=False):
    """Algorithmic operations and state cells of one run of the plan, from
    the instrumented kernels (same search, same evaluations)."""
    cplan = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=False, count_work=True,
                                                     **dict(kw, full_decode=full)), stream)
    cplan.run(stream)
    cres = cplan.results(stream, orders=False, trajectory=False)
    cplan.close()
    assert cres["total_evaluations"] == evals
    return cres["total_work"], cres["total_cells"]


def full_decode_leg(rcpsp, gi, kw, stream, evals):
    """The headline plan with prefix reuse off: every candidate decoded from
    its first position, as the method states it.  One warm-up and one timed
    graph replay, an event-timed run for the kernel's launch time, and a
    counting run for its work; same search and results."""
    import torch
    plan = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=False, **dict(kw, full_decode=True)), stream)
    cfg = plan.config
    plan.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = plan.results(stream, orders=False, trajectory=False)
    assert r["total_evaluations"] == evals
    timed = plan.run_timed(stream)
    plan.close()
    n_launch = cfg["iteration_launches"]
    avg_ms = timed["iteration_ms"] / n_launch
    work, cells = count_work(rcpsp, gi, kw, stream, evals, full=True)
    achieved = (work / n_launch) / (avg_ms * 1e-3)
    lds_b = lds_bytes(work, cells, cfg["eval"], lds_words(gi.info), cfg["finish_bits"])
    out = dict(value=evals / dt, unit="evals/s", ms_per_step=dt * 1e3, ops_per_evaluation=work / evals,
               roofline=dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_INT_OPS / 1e12, unit="Tops/s",
                             frac=achieved / PEAK_INT_OPS, avg_launch_ms=avg_ms,
                             lds=dict(achieved=(lds_b / n_launch) / (avg_ms * 1e-3) / 1e12,
                                      peak=PEAK_LDS_BYTES / 1e12, unit="TB/s",
                                      frac=(lds_b / n_launch) / (avg_ms * 1e-3) / PEAK_LDS_BYTES,
                                      bytes_per_evaluation=lds_b / evals)))
    log("full decode", out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--decoder", choices=["auto", "time", "capacity"], default="auto")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--profile-len", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--full-decode", action="store_true", help="decode every candidate from position 0")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for HBM counter runs: one elementwise kernel over 1 GiB (read 1 GiB, write 1 GiB), "
                         "then one run of the headline plan")
    ap.add_argument("--batch-steps", type=int, default=1)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-large", action="store_true", help="skip the large-instance leg")
    ap.add_argument("--no-hosted", action="store_true", help="skip the heterogeneous-model leg")
    ap.add_argument("--convergence", type=int, default=3, metavar="SEEDS",
                    help="convergence study with this many seeds per point (0 = off; the paper used 50)")
    ap.add_argument("--reselect", type=int, default=0, metavar="PERIOD",
                    help="also run periodic decoder re-selection with this period (two periods)")
    ap.add_argument("--serve-rate", type=float, default=SERVE["rate"])
    ap.add_argument("--serve-seconds", type=float, default=SERVE["measure_s"])
    ap.add_argument("--serve-big-threads", type=int, default=512,
                    help="threads per search of the 300-activity serving class")
    ap.add_argument("--serve-reduced-rate", type=float, default=SERVE["reduced_rate"],
                    help="second serving run at this arrival rate (0 = off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the searches would shard across "
              "GPUs by instance or by search block, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_04556_amd import rcpsp, synth

    if not torch.cuda.is_available():
        log("no GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    inst = synth.instance_120_rs30()
    dec_req = {"auto": rcpsp.EVAL_AUTO, "time": rcpsp.EVAL_TIME, "capacity": rcpsp.EVAL_CAPACITY}[args.decoder]
    gi = rcpsp.Instance(inst, eval=dec_req)
    info = gi.info
    kw = dict(WORKLOAD, threads=args.threads, profile_len=args.profile_len, full_decode=args.full_decode,
              eval=dec_req)
    params = rcpsp.search_params(record_trajectory=False, **kw)
    tuning = None
    if not args.no_tune:
        # decoder and launch shape chosen per instance before the search (outside the timed region)
        t0 = time.perf_counter()
        params, tuning = rcpsp.autotune(gi, params, trial_iterations=10, stream=stream)
        tuning["seconds"] = time.perf_counter() - t0
        log("autotune", tuning)
    kw.update(eval=params.eval, threads=params.threads, profile_len=params.profile_len, lanes=params.lanes,
              lane_profile=params.lane_profile)

    if args.traffic_probe:
        # calibration kernel of known traffic, then the plan's kernels once
        x = torch.zeros(TRAFFIC_PROBE_BYTES // 4, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.bitwise_not(x, out=y)
        torch.cuda.synchronize()
        del x, y
        plan = rcpsp.SearchPlan(gi, params, stream)
        plan.run(stream)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": TRAFFIC_PROBE_BYTES, "plan": plan.config}),
              flush=True)
        plan.close()
        return

    plan = rcpsp.SearchPlan(gi, params, stream)
    cfg = plan.config
    dec = cfg["eval"]
    log("plan", cfg, "info", info)
    for _ in range(args.warmup):
        plan.run(stream)
    torch.cuda.synchronize()
    res = plan.results(stream, orders=False, trajectory=False) if args.warmup > 0 else None

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res2 = plan.results(stream, orders=False, trajectory=False)
    # every run of a plan is the same search: its results never change
    res = res if res is not None else res2
    evals = res["total_evaluations"]
    assert res2["total_evaluations"] == evals and res2["global_best"] == res["global_best"]
    ms_step = dt / args.steps * 1e3
    value = evals * args.steps / dt
    log(f"steps {args.steps}: {ms_step:.2f} ms/step, {evals} evaluations/step, {value:.4g} evals/s")

    # dominant kernel: the iteration kernel; device time from HIP events on the launch stream
    timed = plan.run_timed(stream)
    n_launch = cfg["iteration_launches"]
    avg_ms = timed["iteration_ms"] / n_launch
    log("event-timed run", timed, "iteration launches", n_launch, f"avg {avg_ms:.4f} ms")
    # algorithmic work of the same (deterministic) run, from the instrumented
    # kernels: the decodes this plan makes (shared prefixes once per wave,
    # each candidate from its first swapped position) ...
    work, cells = count_work(rcpsp, gi, kw, stream, evals)
    achieved = (work / n_launch) / (avg_ms * 1e-3)
    lds_b = lds_bytes(work, cells, dec, lds_words(info), cfg["finish_bits"])
    lds_rate = (lds_b / n_launch) / (avg_ms * 1e-3)
    log(f"work {work} ops ({work / evals:.1f} per evaluation), achieved {achieved / 1e12:.3f} Tops/s, "
        f"LDS {lds_rate / 1e12:.3f} TB/s")
    # ... and the method's work per evaluation: every candidate decoded from
    # its first position (prefix reuse off), timed and counted on its own
    full = full_decode_leg(rcpsp, gi, kw, stream, evals) if not args.full_decode else None

    cp = info["critical_path"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "plain: 480 seeded searches x 1000 iterations on one 120-activity instance "
                        "(4 resources, durations 1..10, RF 0.5, RS 0.3), swap range 20, tabu list 329, "
                        "working set 16, phi_max 3, phi_steps 20, one graph replay per step",
            "decoder": {1: "time-indexed", 2: "capacity-indexed"}[dec],
            "threads_per_search": cfg["threads"],
            "profile_len": cfg["profile_len"],
            "register_profile": bool(cfg["register_profile"]),
            "lds_bytes": cfg["lds_bytes"],
            "evaluations_per_step": evals,
            "best_makespan": res["global_best"],
            "critical_path": cp,
            "cpm_dev_pct": 100.0 * (res["global_best"] - cp) / cp,
            "overflow_decodes_per_step": res["overflow_decodes"],
            "prefix_reuse": not args.full_decode,
            "autotune": tuning,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_INT_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved / PEAK_INT_OPS,
            "traffic": measured_traffic(cfg),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "kernel": "k_search (iteration kernel)",
            "avg_launch_ms": avg_ms,
            "ops_per_evaluation": work / evals,
            "ops_basis": "decodes the timed kernel runs (shared prefix once per wave, each candidate from its "
                         "first swapped position; int32 lane operations of Algs. 5-7)",
            "method_ops_per_evaluation": full["ops_per_evaluation"] if full else work / evals,
            "launches_per_step": n_launch,
            "lds": {"achieved": lds_rate / 1e12, "peak": PEAK_LDS_BYTES / 1e12, "unit": "TB/s",
                    "frac": lds_rate / PEAK_LDS_BYTES, "bytes_per_evaluation": lds_b / evals,
                    "basis": "4 B x dwords per packed profile unit per cell touched (all resources of a time "
                             "unit), one finish time per other operation"},
            "counters": counter_fractions(cfg, avg_ms),
        },
        "full_decode": full,
        "prefix_reuse_speedup": (value / full["value"]) if full else None,
        "batched": None,
        "hosted": None,
        "serving": None,
        "serving_reduced": None,
        "large": None,
        "cpu_baseline": None,
    }
    plan.close()
    if not args.no_hosted:
        out["hosted"] = hosted_leg(rcpsp, gi, gi.info["eval"], stream)
    if args.convergence > 0:
        # the default is a short study (1..480 searches, 3 seeds); the paper's
        # figure averages 50 runs (--convergence 50, about 10 minutes)
        short = args.convergence < 10
        out["convergence"] = convergence_leg(rcpsp, gi, gi.info["eval"], stream, args.convergence,
                                             searches=(1, 4, 16, 64, 480) if short else (1, 4, 16, 64, 256, 480))
    if args.reselect > 0:
        ti = kw["eval"] == rcpsp.EVAL_TIME
        out["reselect"] = reselect_leg(rcpsp, gi, stream, args.reselect, max(1, args.reselect // 100),
                                       kw["threads"] if ti else 0, kw["profile_len"] if ti else 0)
    if not args.no_batch:
        out["batched"] = batched_leg(rcpsp, synth, stream, args.batch_steps, 0)
    if not args.no_large:
        out["large"] = large_leg(rcpsp, synth, stream, 1)
    if not args.no_serve:
        out["serving"] = serving_leg(rcpsp, synth, stream, args.serve_rate, SERVE["warmup_s"], args.serve_seconds,
                                     args.serve_big_threads)
        if args.serve_reduced_rate > 0:
            # the 300-activity requests cost ~1.5 GPUs at 2000 requests/s (16
            # searches x ~4,750 evaluations per iteration each): a rate at
            # which they still get their first iteration within the budget
            out["serving_reduced"] = serving_leg(rcpsp, synth, stream, args.serve_reduced_rate, SERVE["warmup_s"],
                                                 SERVE["reduced_measure_s"], args.serve_big_threads)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, dec)
        log("cpu baseline", out["cpu_baseline"])
        out["cpu_parallel"] = cpu_parallel(inst, dec)
        log("cpu parallel", out["cpu_parallel"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
