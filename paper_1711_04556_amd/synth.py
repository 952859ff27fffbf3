"""Seeded synthetic RCPSP instances (input generation only).

This module produces plain integer arrays describing project instances in the
form of the problem statement (Section 2): activities 0..N-1 with dummies 0 and
N-1 of zero duration, M renewable resources with capacities R_k, requests
r_{i,k} <= R_k and a precedence DAG given as successor lists (the "Successors"
column of Table 1).  It holds none of the search method's arithmetic: no
schedule decoding, no neighbourhood, no tabu logic.  Both the CPU oracle tests
and the GPU tests draw their inputs from here.

The paper measured on the PSPLIB J30..J120 sets, which are not available here;
these instances stand in for their shapes (4 resources, 30..120 activities,
about 1.8 arcs per node, durations 1..10, requests 1..10, resource factor and
resource strength in PSPLIB-like ranges).  No PSPLIB instance is reproduced.

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode:
    key   = mix64(seed + (stream + 1) * GAMMA)
    x_i   = mix64(key + (i + 1) * GAMMA)          (i = 0, 1, 2, ...)
all arithmetic modulo 2**64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


class Stream:
    """Counter-based SplitMix64 stream (seed, stream) -> x_0, x_1, ..."""

    def __init__(self, seed: int, stream: int = 0):
        self.key = mix64((seed + (stream + 1) * GAMMA) & M64)
        self.ctr = 0

    def next(self) -> int:
        self.ctr += 1
        return mix64((self.key + self.ctr * GAMMA) & M64)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by the multiply-shift map of the high word."""
        return ((self.next() >> 32) * n) >> 32


@dataclass
class Instance:
    """A project: N activities (incl. dummies 0 and N-1), M resources."""
    n: int                      # N, including the two dummies
    m: int                      # M
    duration: List[int]         # [N]
    capacity: List[int]         # [M]
    request: List[int]          # [N*M], row-major: request[i*M + k]
    succ: List[List[int]]       # successor lists, ascending
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def succ_off(self) -> List[int]:
        off = [0]
        for s in self.succ:
            off.append(off[-1] + len(s))
        return off

    @property
    def succ_flat(self) -> List[int]:
        return [j for s in self.succ for j in s]

    @property
    def n_arcs(self) -> int:
        return sum(len(s) for s in self.succ)

    def r(self, i: int, k: int) -> int:
        return self.request[i * self.m + k]


def _es_peak_usage(n_tot: int, m: int, d: Sequence[int], succ: Sequence[Sequence[int]],
                   req: Sequence[int]) -> List[int]:
    """Peak per-period usage of each resource in the precedence-only
    earliest-start schedule.  Used only to set capacities from the resource
    strength (Kolisch, Sprecher & Drexl, Management Science 41(10), 1995);
    activity ids are topologically ordered by construction."""
    es = [0] * n_tot
    for i in range(n_tot):
        for j in succ[i]:
            es[j] = max(es[j], es[i] + d[i])
    horizon = max(es[i] + d[i] for i in range(n_tot)) + 1
    peak = [0] * m
    for k in range(m):
        use = [0] * horizon
        for i in range(n_tot):
            rik = req[i * m + k]
            if rik:
                for t in range(es[i], es[i] + d[i]):
                    use[t] += rik
        peak[k] = max(use) if use else 0
    return peak


def generate(n: int, m: int = 4, d_max: int = 10, rf: float = 0.5, rs: Optional[float] = 0.5,
             cap_range: Optional[Tuple[int, int]] = None, seed: int = 1, r_max: int = 10,
             name: str = "") -> Instance:
    """Deterministic synthetic instance with n non-dummy activities.

    - d_i = 1 + x mod d_max
    - successor count c in {1,1,2,2,3}[x mod 5] (mean 1.8), capped at n - i,
      drawn without replacement from {i+1..n} (acyclic by topological index)
    - 0 -> i for every i without predecessor, i -> N-1 for every i without successor
    - r_ik = 1 + (x >> 32) mod r_max with probability rf (x mod 100 < 100 rf), else 0
    - capacities: resource strength rs (K_min + round(rs (K_max - K_min))) or,
      if cap_range is given, uniform in the range (raised to max_i r_ik)
    """
    rng = Stream(seed, 0)
    N = n + 2
    d = [0] * N
    for i in range(1, n + 1):
        d[i] = 1 + rng.next() % d_max
    succ = [set() for _ in range(N)]
    for i in range(1, n + 1):
        c = (1, 1, 2, 2, 3)[rng.next() % 5]
        span = n - i
        c = min(c, span)
        cand = list(range(i + 1, n + 1))
        for j in range(c):
            k = j + rng.next() % (span - j)
            cand[j], cand[k] = cand[k], cand[j]
            succ[i].add(cand[j])
    has_pred = [False] * N
    for i in range(1, n + 1):
        for j in succ[i]:
            has_pred[j] = True
    for i in range(1, n + 1):
        if not has_pred[i]:
            succ[0].add(i)
        if not succ[i]:
            succ[i].add(N - 1)
    req = [0] * (N * m)
    rf_pct = int(round(rf * 100))
    for i in range(1, n + 1):
        for k in range(m):
            x = rng.next()
            if x % 100 < rf_pct:
                req[i * m + k] = 1 + (x >> 32) % r_max
    kmin = [max(req[i * m + k] for i in range(N)) for k in range(m)]
    cap = [0] * m
    if cap_range is not None:
        lo, hi = cap_range
        for k in range(m):
            cap[k] = max(lo + rng.next() % (hi - lo + 1), kmin[k], 1)
    else:
        succ_l = [sorted(s) for s in succ]
        peak = _es_peak_usage(N, m, d, succ_l, req)
        rs_pct = int(round(rs * 100))
        for k in range(m):
            cap[k] = max(kmin[k] + (rs_pct * (peak[k] - kmin[k]) + 50) // 100, 1)
    inst = Instance(n=N, m=m, duration=d, capacity=cap, request=req,
                    succ=[sorted(s) for s in succ], name=name or f"G({n},{m},{d_max},{rf},{rs},{cap_range},{seed})")
    inst.meta = dict(n_real=n, d_max=d_max, rf=rf, rs=rs, cap_range=cap_range, seed=seed)
    return inst


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_instance_30(seed: int = 1) -> Instance:
    """30 activities, 4 resources, durations 1..10, RF 0.5, RS 0.5."""
    return generate(30, 4, 10, 0.5, rs=0.5, seed=seed, name=f"g30_rs50_s{seed}")


def instance_120_rs30(seed: int = 2) -> Instance:
    """120 activities, 4 resources, durations 1..10, RF 0.5, RS 0.3."""
    return generate(120, 4, 10, 0.5, rs=0.3, seed=seed, name=f"g120_rs30_s{seed}")


def mixed_batch(count: int = 1024, base_seed: int = 3000) -> List[Instance]:
    """Mixed sizes {30,60,120}[i mod 3], 4 resources, RF in {.25,.5,.75,1},
    RS in {.2,...,.7} (discrete uniform), seed base_seed + i."""
    out = []
    for i in range(count):
        s = Stream(base_seed + i, 1)
        rf = (0.25, 0.5, 0.75, 1.0)[s.next() % 4]
        rs = (0.2, 0.3, 0.4, 0.5, 0.6, 0.7)[s.next() % 6]
        n = (30, 60, 120)[i % 3]
        out.append(generate(n, 4, 10, rf, rs=rs, seed=base_seed + i, name=f"mix{i}_n{n}"))
    return out


def large_batch(count: int = 256, base_seed: int = 4000) -> List[Instance]:
    """300 activities, 8 resources, durations 1..20, capacities 10..60."""
    return [generate(300, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=base_seed + i,
                     name=f"big{i}") for i in range(count)]


SERVING_SIZES = (30, 60, 120, 300)


def serving_pool(per_size: int = 256, base_seed: int = 5000) -> dict:
    """Instances for the serving workload, per size in SERVING_SIZES: 30, 60
    and 120 activities as in mixed_batch (4 resources, RF and RS varied), 300
    with the large generator (8 resources, durations 1..20, capacities
    10..60).  Entry j of size index s has seed base_seed + 4 j + s."""
    out = {}
    for si, n in enumerate(SERVING_SIZES):
        lst = []
        for j in range(per_size):
            seed = base_seed + 4 * j + si
            if n == 300:
                lst.append(generate(300, 8, 20, 0.5, rs=None, cap_range=(10, 60), seed=seed, name=f"srv{seed}"))
            else:
                st = Stream(seed, 1)
                rf = (0.25, 0.5, 0.75, 1.0)[st.next() % 4]
                rs = (0.2, 0.3, 0.4, 0.5, 0.6, 0.7)[st.next() % 6]
                lst.append(generate(n, 4, 10, rf, rs=rs, seed=seed, name=f"srv{seed}"))
        out[n] = lst
    return out


def serving_arrivals(rate: float, duration_s: float, seed: int = 5) -> List[tuple]:
    """Open-loop arrivals over [0, duration_s): exponential inter-arrival
    times of mean 1/rate and a size index uniform over SERVING_SIZES, from
    streams 0 and 1 of `seed`.  Returns [(time_s, size_index)]."""
    a, z = Stream(seed, 0), Stream(seed, 1)
    t, out = 0.0, []
    while True:
        u = ((a.next() >> 11) + 0.5) / float(1 << 53)
        t += -math.log(u) / rate
        if t >= duration_s:
            return out
        out.append((t, z.below(len(SERVING_SIZES))))


def table1_instance() -> Instance:
    """The example instance of Table 1 (Section 2.2) with capacities (6, 6)
    (the text states a maximal capacity of 6 for both resources)."""
    d = [0, 4, 3, 5, 5, 3, 2, 4, 2, 3, 4, 0]
    r = [(0, 0), (5, 3), (2, 1), (3, 2), (2, 3), (3, 4), (4, 1), (2, 2), (4, 5), (1, 2), (2, 2), (0, 0)]
    succ = [[1, 2], [3, 6], [4, 5], [5, 10], [7], [8, 9], [7, 9], [8, 10], [11], [11], [11], []]
    req = [x for pair in r for x in pair]
    return Instance(n=12, m=2, duration=d, capacity=[6, 6], request=req, succ=succ, name="table1")


def random_tiny(seed: int, n_real: int = 5, m: int = 2, d_max: int = 4, r_max: int = 3,
                arc_p: int = 35) -> Instance:
    """Small random instance for brute-force checks (n_real <= 6).  Arcs i->j
    for i<j with probability arc_p percent; capacities between max request
    and total request."""
    rng = Stream(seed, 7)
    N = n_real + 2
    d = [0] + [1 + rng.next() % d_max for _ in range(n_real)] + [0]
    succ = [set() for _ in range(N)]
    for i in range(1, n_real + 1):
        for j in range(i + 1, n_real + 1):
            if rng.next() % 100 < arc_p:
                succ[i].add(j)
    has_pred = [False] * N
    for i in range(1, n_real + 1):
        for j in succ[i]:
            has_pred[j] = True
    for i in range(1, n_real + 1):
        if not has_pred[i]:
            succ[0].add(i)
        if not succ[i]:
            succ[i].add(N - 1)
    req = [0] * (N * m)
    for i in range(1, n_real + 1):
        for k in range(m):
            req[i * m + k] = rng.next() % (r_max + 1)
    cap = []
    for k in range(m):
        lo = max(1, max(req[i * m + k] for i in range(N)))
        hi = max(lo, sum(req[i * m + k] for i in range(N)))
        cap.append(lo + rng.next() % (hi - lo + 1))
    return Instance(n=N, m=m, duration=d, capacity=cap, request=req,
                    succ=[sorted(s) for s in succ], name=f"tiny{seed}")


def random_feasible_order(inst: Instance, seed: int) -> List[int]:
    """A random precedence-feasible activity list (random topological order
    with 0 first and N-1 last); input generation for parity tests."""
    rng = Stream(seed, 11)
    N = inst.n
    indeg = [0] * N
    for i in range(N):
        for j in inst.succ[i]:
            indeg[j] += 1
    ready = [i for i in range(N) if indeg[i] == 0]
    out = []
    while ready:
        if len(ready) > 1 and N - 1 in ready:
            ready.remove(N - 1)
            pick = ready.pop(rng.below(len(ready)))
            ready.append(N - 1)
        else:
            pick = ready.pop(rng.below(len(ready)))
        out.append(pick)
        for j in inst.succ[pick]:
            indeg[j] -= 1
            if indeg[j] == 0:
                ready.append(j)
    return out
