"""Python access to the plain C oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product library under paper_1711_04556_amd never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rcpsp_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

TIME = 1
CAPACITY = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "rcpsp_oracle.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        i32p, u8p, i64p, u32p = P(ctypes.c_int), P(ctypes.c_uint8), P(ctypes.c_int64), P(ctypes.c_uint32)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, i32p, i32p]
        L.orc_free.argtypes = [ctypes.c_void_p]
        for f in ("orc_n", "orc_horizon", "orc_critical_path"):
            getattr(L, f).argtypes = [ctypes.c_void_p]
            getattr(L, f).restype = ctypes.c_int
        L.orc_levels.argtypes = [ctypes.c_void_p, i32p]
        for f in ("orc_decode_time", "orc_decode_time_alg5", "orc_decode_capacity"):
            getattr(L, f).argtypes = [ctypes.c_void_p, i32p, i32p]
            getattr(L, f).restype = ctypes.c_int
        L.orc_decode.argtypes = [ctypes.c_void_p, ctypes.c_int, i32p, i32p]
        L.orc_capacity_update.argtypes = [ctypes.c_int, i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p]
        L.orc_work_counters.argtypes = [i64p]
        L.orc_count_potential.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_is_feasible_order.argtypes = [ctypes.c_void_p, i32p]
        L.orc_move_feasible.argtypes = [ctypes.c_void_p, i32p, ctypes.c_int, ctypes.c_int]
        L.orc_evaluate_neighbourhood.argtypes = [ctypes.c_void_p, ctypes.c_int, i32p, ctypes.c_int, u8p,
                                                 ctypes.c_int, i32p, i32p]
        L.orc_stl_add.argtypes = [ctypes.c_int, i32p, i32p, i32p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_stl_check.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_rng.restype = ctypes.c_uint64
        L.orc_rng.argtypes = [ctypes.c_uint64] * 3
        L.orc_rng_below.restype = ctypes.c_uint32
        L.orc_rng_below.argtypes = [ctypes.c_uint64] * 3 + [ctypes.c_uint32]
        L.orc_initial_order.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, i32p]
        L.orc_decay_table.argtypes = [u32p, ctypes.c_int]
        L.orc_iterations_assigned.argtypes = [ctypes.c_int] * 4
        L.orc_tabu_search.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_tabu_search.restype = ctypes.c_int
        L.orc_fbi.argtypes = [ctypes.c_void_p, ctypes.c_int, i32p]
        L.orc_fbi.restype = ctypes.c_int
        _lib = L
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a: np.ndarray, ct=ctypes.c_int):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OrcParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_int), ("tabu_len", ctypes.c_int), ("iterations", ctypes.c_int),
                ("searches", ctypes.c_int), ("elite", ctypes.c_int), ("phi_max", ctypes.c_int),
                ("phi_steps", ctypes.c_int), ("decoder", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("i_block", ctypes.c_int), ("fbi", ctypes.c_int),
                ("decoder_of_iteration", ctypes.POINTER(ctypes.c_int32)),
                ("exchange_every", ctypes.c_int), ("round_log", ctypes.POINTER(ctypes.c_int32)),
                ("round_log_cap", ctypes.c_int)]


class OrcResults(ctypes.Structure):
    _fields_ = [("best_makespan", ctypes.c_void_p), ("best_order", ctypes.c_void_p),
                ("iterations_done", ctypes.c_void_p), ("evaluations", ctypes.c_void_p),
                ("trajectory", ctypes.c_void_p), ("elite_makespan", ctypes.c_void_p),
                ("elite_order", ctypes.c_void_p)]


class Oracle:
    """One project instance held by the oracle."""

    def __init__(self, inst):
        L = lib()
        self.inst = inst
        self.n = inst.n
        self.m = inst.m
        self._d = _i32(inst.duration)
        self._R = _i32(inst.capacity)
        self._r = _i32(inst.request)
        self._so = _i32(inst.succ_off)
        self._s = _i32(inst.succ_flat if inst.n_arcs else [0])
        self.h = L.orc_create(inst.n, inst.m, _p(self._d), _p(self._R), _p(self._r), _p(self._so), _p(self._s))
        if not self.h:
            raise ValueError("oracle rejected the instance (not a DAG?)")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_free(self.h)
            self.h = None

    @property
    def horizon(self) -> int:
        return lib().orc_horizon(self.h)

    @property
    def critical_path(self) -> int:
        return lib().orc_critical_path(self.h)

    def levels(self) -> List[int]:
        out = np.zeros(self.n, dtype=np.int32)
        lib().orc_levels(self.h, _p(out))
        return out.tolist()

    def decode(self, order: Sequence[int], decoder: int = TIME, starts: bool = False):
        o = _i32(order)
        s = np.zeros(self.n, dtype=np.int32)
        fn = {TIME: lib().orc_decode_time, CAPACITY: lib().orc_decode_capacity, 5: lib().orc_decode_time_alg5}[decoder]
        c = fn(self.h, _p(o), _p(s))
        return (c, s.tolist()) if starts else c

    def work_counters(self) -> List[int]:
        out = np.zeros(4, dtype=np.int64)
        lib().orc_work_counters(_p(out, ctypes.c_int64))
        return out.tolist()

    def work_reset(self) -> None:
        lib().orc_work_reset()

    def is_feasible_order(self, order) -> bool:
        return bool(lib().orc_is_feasible_order(self.h, _p(_i32(order))))

    def move_feasible(self, order, u: int, v: int) -> bool:
        return bool(lib().orc_move_feasible(self.h, _p(_i32(order)), u, v))

    def count_potential(self, delta: int) -> int:
        return lib().orc_count_potential(self.n, delta)

    def evaluate_neighbourhood(self, order, delta: int, decoder: int = TIME, tabu: Optional[np.ndarray] = None,
                               aspiration: int = 2 ** 31 - 1):
        P = self.count_potential(delta)
        mk = np.zeros(max(P, 1), dtype=np.int32)
        best = np.zeros(4, dtype=np.int32)
        tb = None
        if tabu is not None:
            tb = np.ascontiguousarray(np.asarray(tabu, dtype=np.uint8).reshape(self.n * self.n))
        lib().orc_evaluate_neighbourhood(self.h, decoder, _p(_i32(order)), delta,
                                         _p(tb, ctypes.c_uint8) if tb is not None else None,
                                         aspiration, _p(mk), _p(best))
        return mk[:P], best.tolist()

    def fbi(self, order: Sequence[int], decoder: int = TIME):
        """Forward-backward improvement of an activity list: (improved list, makespan)."""
        o = _i32(order).copy()
        c = lib().orc_fbi(self.h, decoder, _p(o))
        return o.tolist(), c

    def initial_order(self, seed: int, stream: int) -> List[int]:
        out = np.zeros(self.n, dtype=np.int32)
        lib().orc_initial_order(self.h, seed, stream, _p(out))
        return out.tolist()

    def tabu_search(self, delta: int, tabu_len: int, iterations: int, searches: int = 1, elite: int = 0,
                    phi_max: int = 3, phi_steps: int = 20, decoder: int = TIME, seed: int = 1,
                    trajectory: bool = True, i_block: int = 0, fbi: bool = False,
                    decoder_of_iteration: Optional[Sequence[int]] = None, exchange_every: int = 1,
                    round_log: bool = False) -> dict:
        """i_block: eq. 8's iteration allowance when it differs from the
        iterations run (a search cut short by a time budget); 0 = iterations.
        fbi: forward-backward improvement of every second initial solution.
        decoder_of_iteration: per iteration, the decoder of its decodes
        (periodic re-selection); set-up decodes keep `decoder`.
        exchange_every: iterations between exchange rounds.
        round_log: also return out["rounds"], the state after every exchange
        round: a list of dicts with per-record C, IC, reads, W and per-search
        slot, I_assigned, C_read, C_cur, C_best."""
        B, N = searches, self.n
        out = dict(best_makespan=np.zeros(B, np.int32), best_order=np.zeros((B, N), np.int32),
                   iterations_done=np.zeros(B, np.int32), evaluations=np.zeros(B, np.int64),
                   trajectory=np.zeros((B, iterations, 4), np.int32) if trajectory else None,
                   elite_makespan=np.zeros(max(elite, 1), np.int32),
                   elite_order=np.zeros((max(elite, 1), N), np.int32))
        sched = None
        if decoder_of_iteration is not None:
            sched = _i32(list(decoder_of_iteration)).copy()
            assert len(sched) == iterations and set(sched.tolist()) <= {TIME, CAPACITY}
        stride = elite * (3 + N) + 5 * B
        cap = (iterations // max(exchange_every, 1) + 1) if (round_log and elite > 0) else 0
        log = np.zeros(max(cap * stride, 1), np.int32)
        prm = OrcParams(delta, tabu_len, iterations, searches, elite, phi_max, phi_steps, decoder, seed, i_block,
                        int(fbi), _p(sched) if sched is not None else None, exchange_every,
                        _p(log) if cap else None, cap)
        res = OrcResults(*[out[k].ctypes.data if out[k] is not None else None for k in
                           ("best_makespan", "best_order", "iterations_done", "evaluations", "trajectory",
                            "elite_makespan", "elite_order")])
        rounds = lib().orc_tabu_search(self.h, ctypes.byref(prm), ctypes.byref(res))
        out["elite_makespan"] = out["elite_makespan"][:elite]
        out["elite_order"] = out["elite_order"][:elite]
        if round_log:
            out["rounds"] = []
            for r in range(min(rounds, cap)):
                row = log[r * stride:(r + 1) * stride]
                recs = row[:elite * (3 + N)].reshape(elite, 3 + N)
                srch = row[elite * (3 + N):].reshape(B, 5)
                out["rounds"].append(dict(C=recs[:, 0].copy(), IC=recs[:, 1].copy(), reads=recs[:, 2].copy(),
                                          W=recs[:, 3:].copy(), slot=srch[:, 0].copy(),
                                          I_assigned=srch[:, 1].copy(), C_read=srch[:, 2].copy(),
                                          C_cur=srch[:, 3].copy(), C_best=srch[:, 4].copy()))
        return out


def capacity_update(R: int, c: Sequence[int], r: int, d: int, s: int):
    """Alg. 4 on one resource array; returns (new array, residual effort)."""
    arr = _i32(list(c)).copy()
    was = np.zeros(max(R, 1), dtype=np.int32)
    res = lib().orc_capacity_update(R, _p(arr), r, d, s, _p(was))
    return arr.tolist(), res


def stl_add(ring_u, ring_v, widx: List[int], cache: np.ndarray, n: int, u: int, v: int):
    """Alg. 3 on numpy storage (ring_u, ring_v int32 arrays; widx a 1-element int32 array)."""
    lib().orc_stl_add(len(ring_u), _p(ring_u), _p(ring_v), _p(widx), _p(cache, ctypes.c_uint8), n, u, v)


def stl_check(cache: np.ndarray, n: int, u: int, v: int) -> bool:
    return bool(lib().orc_stl_check(_p(cache, ctypes.c_uint8), n, u, v))


def mix64(z: int) -> int:
    return lib().orc_mix64(z)


def rng(seed: int, stream: int, i: int) -> int:
    return lib().orc_rng(seed, stream, i)


def decay_table() -> List[int]:
    n = lib().orc_decay_table(None, 0)
    out = np.zeros(n, dtype=np.uint32)
    lib().orc_decay_table(_p(out, ctypes.c_uint32), n)
    return out.tolist()


def iterations_assigned(i_block: int, c_k: int, c_star: int, ic_k: int) -> int:
    return lib().orc_iterations_assigned(i_block, c_k, c_star, ic_k)
