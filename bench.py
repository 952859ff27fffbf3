"""Benchmark: SSGS neighbour evaluations per second of the tabu search on one
MI355X, for 480 seeded searches x 1000 iterations on one 120-activity
instance (4 resources, resource strength 0.3, swap range 20, tabu list 329,
working set of 16 records, phi_max 3, phi_steps 20).

One step = one whole search run from its initial state (every iteration of
every search plus the working-set exchange rounds), replayed from a captured
HIP graph; the instance and all search state are resident in HBM.

Prints one JSON line on stdout (details on stderr)."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSGS neighbour evals/s (batched vs plain) at bit-exact makespan; p50/p99 latency"
PEAK_INT_OPS = 256 * 64 * 2.4e9      # 256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer op per lane-cycle

WORKLOAD = dict(swap_range=20, tabu_len=329, iterations=1000, searches=480, elite=16, phi_max=3, phi_steps=20,
                seed=2)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(inst, decoder, iters=2):
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
    kw.update(eval=params.eval, threads=params.threads, profile_len=params.profile_len)

    plan = rcpsp.SearchPlan(gi, params, stream)
    cfg = plan.config
    dec = cfg["eval"]
    log("plan", cfg, "info", info)
    for _ in range(args.warmup):
        plan.run(stream)
    torch.cuda.synchronize()
    res = plan.results(stream, orders=False, trajectory=False)
    evals = res["total_evaluations"]

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res2 = plan.results(stream, orders=False, trajectory=False)
    assert res2["total_evaluations"] == evals and res2["global_best"] == res["global_best"]
    ms_step = dt / args.steps * 1e3
    value = evals * args.steps / dt
    log(f"steps {args.steps}: {ms_step:.2f} ms/step, {evals} evaluations/step, {value:.4g} evals/s")

    # dominant kernel: the iteration kernel; device time from HIP events on the launch stream
    timed = plan.run_timed(stream)
    n_launch = cfg["iteration_launches"]
    avg_ms = timed["iteration_ms"] / n_launch
    log("event-timed run", timed, "iteration launches", n_launch, f"avg {avg_ms:.4f} ms")
    # algorithmic operations of the same (deterministic) run, from the instrumented kernels
    cplan = rcpsp.SearchPlan(gi, rcpsp.search_params(record_trajectory=False, count_work=True, **kw), stream)
    cplan.run(stream)
    cres = cplan.results(stream, orders=False, trajectory=False)
    assert cres["total_evaluations"] == evals
    work = cres["total_work"]
    cplan.close()
    achieved = (work / n_launch) / (avg_ms * 1e-3)
    log(f"work {work} ops ({work / evals:.1f} per evaluation), achieved {achieved / 1e12:.3f} Tops/s")

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
            "traffic": None,
            "kernel": "k_search (iteration kernel)",
            "avg_launch_ms": avg_ms,
            "ops_per_evaluation": work / evals,
            "launches_per_step": n_launch,
        },
        "cpu_baseline": None,
    }
    plan.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, dec)
        log("cpu baseline", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
