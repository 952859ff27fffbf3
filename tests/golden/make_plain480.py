"""Writes tests/golden/plain480_ti.json: the oracle's results for the
benchmarked workload, so that GPU runs of it can be compared with the oracle
at full length.

Workload: one 120-activity instance (4 resources, resource strength 0.3,
instance seed 2), 480 cooperating searches x 1000 iterations, swap range 20,
tabu list 329, working set of 16 records, phi_max 3, phi_steps 20, search
seed 2, time-indexed serial schedule generation (Section 6 main loop with the
exchange rounds of Section 6.1).

Only the oracle runs here (one host thread, about 40 minutes).  The stored
values: every search's best makespan, iterations done and evaluations, the
final working set (makespans and orders), and SHA-256 digests of the int32
trajectory array [480][1000][4] = (u, v, C', C_best) per search and
iteration and of the int32 best-order array [480][122], both little-endian.

    python tests/golden/make_plain480.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1711_04556_amd import synth  # noqa: E402

WORKLOAD = dict(delta=20, tabu_len=329, iterations=1000, searches=480, elite=16, phi_max=3, phi_steps=20, seed=2)
OUT = os.path.join(HERE, "plain480_ti.json")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def main():
    inst = synth.instance_120_rs30(2)
    o = oracle.Oracle(inst)
    w = WORKLOAD
    t0 = time.time()
    r = o.tabu_search(w["delta"], w["tabu_len"], w["iterations"], searches=w["searches"], elite=w["elite"],
                      phi_max=w["phi_max"], phi_steps=w["phi_steps"], decoder=oracle.TIME, seed=w["seed"],
                      trajectory=True)
    dt = time.time() - t0
    out = {
        "source": "oracle/ (tabu_search), written by tests/golden/make_plain480.py",
        "workload": dict(w, instance="synth.instance_120_rs30(2)", decoder="time-indexed"),
        "n": inst.n,
        "critical_path": o.critical_path,
        "best_makespan": r["best_makespan"].tolist(),
        "iterations_done": r["iterations_done"].tolist(),
        "evaluations": [int(x) for x in r["evaluations"]],
        "elite_makespan": r["elite_makespan"].tolist(),
        "elite_order": r["elite_order"].tolist(),
        "trajectory_sha256": digest(r["trajectory"]),
        "best_order_sha256": digest(r["best_order"]),
        "oracle_seconds": round(dt, 1),
    }
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} ({dt:.0f} s)")


if __name__ == "__main__":
    main()
