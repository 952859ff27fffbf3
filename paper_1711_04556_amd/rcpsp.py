"""Python binding of librcpsp (include/rcpsp.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and torch tensors to pointers and status codes to exceptions.  It raises if
the library has not been built or cannot be loaded (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .build import LIB

INT32_MAX = 2 ** 31 - 1

EVAL_AUTO, EVAL_TIME, EVAL_CAPACITY = 0, 1, 2

STATUS = {
    0: "RCPSP_OK", -1: "RCPSP_E_ARG", -2: "RCPSP_E_CYCLE", -3: "RCPSP_E_REQUEST", -4: "RCPSP_E_DUMMY",
    -5: "RCPSP_E_ORDER", -6: "RCPSP_E_BUFFER", -7: "RCPSP_E_NOMEM", -8: "RCPSP_E_DEVICE", -9: "RCPSP_E_TOO_LARGE",
}


class RcpspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class rcpsp_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n", "m", "n_arcs", "horizon", "critical_path", "eval", "min_capacity", "max_capacity", "sum_capacity",
        "field_bits", "avg_capacity_x1000", "avg_duration_x1000", "branch_factor_x1000")]


class rcpsp_move(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("v", ctypes.c_int32), ("makespan", ctypes.c_int32),
                ("n_feasible", ctypes.c_int32)]


class rcpsp_search_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "swap_range", "tabu_len", "iterations", "searches", "elite", "phi_max", "phi_steps", "threads",
        "profile_len", "record_trajectory", "count_work", "full_decode", "eval", "lanes")] + [
        ("seed", ctypes.c_uint64), ("fbi", ctypes.c_int32), ("exchange_every", ctypes.c_int32),
        ("time_budget_us", ctypes.c_int32), ("lane_profile", ctypes.c_int32)]


class rcpsp_tuning(ctypes.Structure):
    _fields_ = [("eval", ctypes.c_int32), ("threads", ctypes.c_int32), ("profile_len", ctypes.c_int32),
                ("trials", ctypes.c_int32), ("lanes", ctypes.c_int32), ("ns_per_evaluation", ctypes.c_double),
                ("register_profile", ctypes.c_int32)]


class rcpsp_search_result(ctypes.Structure):
    _fields_ = [("best_makespan", ctypes.c_void_p), ("best_order", ctypes.c_void_p),
                ("iterations_done", ctypes.c_void_p), ("evaluations", ctypes.c_void_p),
                ("trajectory", ctypes.c_void_p), ("elite_makespan", ctypes.c_void_p),
                ("elite_order", ctypes.c_void_p), ("global_best", ctypes.c_int32),
                ("total_evaluations", ctypes.c_int64), ("overflow_decodes", ctypes.c_int32),
                ("total_work", ctypes.c_int64), ("total_cells", ctypes.c_int64)]


class rcpsp_batch_info(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int32), ("classes", ctypes.c_int32)] + [
        (n, ctypes.c_int32 * 8) for n in ("class_eval", "class_threads", "class_instances", "class_workgroups",
                                          "class_lds_bytes")]


class rcpsp_batch_tuning(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("trials", ctypes.c_int32)] + [
        (n, ctypes.c_int32 * 8) for n in ("group_n", "group_m", "group_members", "group_eval", "group_threads",
                                          "group_lanes")] + [
        ("group_evals_per_s", ctypes.c_double * 8), ("group_register", ctypes.c_int32 * 8)]


class rcpsp_server_params(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("slice_us", ctypes.c_int32), ("arena_bytes", ctypes.c_int64)]


class rcpsp_request_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("best_makespan", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("error", ctypes.c_int32), ("evaluations", ctypes.c_int64), ("submit_ns", ctypes.c_int64),
                ("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64), ("seen_ns", ctypes.c_int64)]


class rcpsp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("slices", ctypes.c_int64), ("busy_ms", ctypes.c_double), ("evaluations", ctypes.c_int64),
                ("resident", ctypes.c_int32), ("queued", ctypes.c_int32), ("arena_used", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("device_clock_mhz", ctypes.c_double)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class rcpsp_decoder_segment(ctypes.Structure):
    _fields_ = [("first_iteration", ctypes.c_int32), ("iterations", ctypes.c_int32), ("eval", ctypes.c_int32),
                ("probe", ctypes.c_int32), ("ms_per_iteration", ctypes.c_float)]


class rcpsp_search_config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "threads", "profile_len", "lds_bytes", "eval", "iteration_launches", "round_launches", "lanes",
        "finish_bits", "register_profile")]


_lib = None


def lib():
    """Load librcpsp.so; raise if it is missing (build it with
    paper_1711_04556_amd.build.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built; run paper_1711_04556_amd.build.build() first")
    L = ctypes.CDLL(LIB)
    vp, i32, i32p, u8p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p
    L.rcpsp_create_instance.argtypes = [i32, i32, i32p, i32p, i32p, i32p, i32p, ctypes.c_int, ctypes.POINTER(vp)]
    L.rcpsp_create_instance.restype = ctypes.c_int
    L.rcpsp_instance_info.argtypes = [vp, ctypes.POINTER(rcpsp_info)]
    L.rcpsp_instance_info.restype = ctypes.c_int
    L.rcpsp_destroy_instance.argtypes = [vp]
    L.rcpsp_destroy_instance.restype = None
    L.rcpsp_evaluate_neighbourhood.argtypes = [vp, i32p, i32, u8p, i32, i32p, i32, i32p,
                                               ctypes.POINTER(rcpsp_move), vp]
    L.rcpsp_evaluate_neighbourhood.restype = ctypes.c_int
    L.rcpsp_evaluate_neighbourhood_noalloc.argtypes = [vp, i32p, i32, u8p, i32, i32p, i32, i32p,
                                                       ctypes.POINTER(rcpsp_move), vp]
    L.rcpsp_evaluate_neighbourhood_noalloc.restype = ctypes.c_int
    L.rcpsp_evaluate_neighbourhood_device.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.rcpsp_evaluate_neighbourhood_device.restype = ctypes.c_int
    L.rcpsp_potential_moves.argtypes = [i32, i32]
    L.rcpsp_potential_moves.restype = i32
    L.rcpsp_search_create.argtypes = [vp, ctypes.POINTER(rcpsp_search_params), vp, ctypes.POINTER(vp)]
    L.rcpsp_search_create.restype = ctypes.c_int
    L.rcpsp_search_run.argtypes = [vp, vp]
    L.rcpsp_search_run.restype = ctypes.c_int
    L.rcpsp_search_run_timed.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    L.rcpsp_search_run_timed.restype = ctypes.c_int
    L.rcpsp_search_results.argtypes = [vp, ctypes.POINTER(rcpsp_search_result), vp]
    L.rcpsp_search_results.restype = ctypes.c_int
    L.rcpsp_search_destroy.argtypes = [vp]
    L.rcpsp_search_destroy.restype = None
    L.rcpsp_search_get_config.argtypes = [vp, ctypes.POINTER(rcpsp_search_config)]
    L.rcpsp_search_get_config.restype = ctypes.c_int
    L.rcpsp_tabu_search.argtypes = [vp, ctypes.POINTER(rcpsp_search_params), ctypes.POINTER(rcpsp_search_result), vp]
    L.rcpsp_tabu_search.restype = ctypes.c_int
    L.rcpsp_tabu_search_hosted.argtypes = [vp, ctypes.POINTER(rcpsp_search_params),
                                           ctypes.POINTER(rcpsp_search_result), vp]
    L.rcpsp_tabu_search_hosted.restype = ctypes.c_int
    L.rcpsp_tabu_search_reselect.argtypes = [vp, ctypes.POINTER(rcpsp_search_params), i32, i32,
                                             ctypes.POINTER(rcpsp_search_result),
                                             ctypes.POINTER(rcpsp_decoder_segment), i32, i32p, vp]
    L.rcpsp_tabu_search_reselect.restype = ctypes.c_int
    L.rcpsp_autotune.argtypes = [vp, ctypes.POINTER(rcpsp_search_params), i32, vp, ctypes.POINTER(rcpsp_search_params),
                                 ctypes.POINTER(rcpsp_tuning)]
    L.rcpsp_autotune.restype = ctypes.c_int
    L.rcpsp_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(rcpsp_search_params), vp,
                                     ctypes.POINTER(vp)]
    L.rcpsp_batch_create.restype = ctypes.c_int
    L.rcpsp_batch_run.argtypes = [vp, vp]
    L.rcpsp_batch_run.restype = ctypes.c_int
    L.rcpsp_batch_run_timed.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.rcpsp_batch_run_timed.restype = ctypes.c_int
    L.rcpsp_batch_results.argtypes = [vp, i32, ctypes.POINTER(rcpsp_search_result), vp]
    L.rcpsp_batch_results.restype = ctypes.c_int
    L.rcpsp_batch_get_info.argtypes = [vp, ctypes.POINTER(rcpsp_batch_info)]
    L.rcpsp_batch_get_info.restype = ctypes.c_int
    L.rcpsp_batch_destroy.argtypes = [vp]
    L.rcpsp_batch_destroy.restype = None
    L.rcpsp_tabu_search_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(rcpsp_search_params),
                                          ctypes.POINTER(rcpsp_search_result), vp]
    L.rcpsp_tabu_search_batch.restype = ctypes.c_int
    L.rcpsp_batch_autotune.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(rcpsp_search_params), i32, i32, vp,
                                       ctypes.POINTER(rcpsp_search_params), ctypes.POINTER(rcpsp_batch_tuning)]
    L.rcpsp_batch_autotune.restype = ctypes.c_int
    L.rcpsp_server_create.argtypes = [ctypes.POINTER(rcpsp_server_params), ctypes.POINTER(vp)]
    L.rcpsp_server_create.restype = ctypes.c_int
    L.rcpsp_server_submit.argtypes = [vp, vp, ctypes.POINTER(rcpsp_search_params), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)]
    L.rcpsp_server_submit.restype = ctypes.c_int
    L.rcpsp_server_poll.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(rcpsp_request_status)]
    L.rcpsp_server_poll.restype = ctypes.c_int
    L.rcpsp_server_results.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(rcpsp_search_result)]
    L.rcpsp_server_results.restype = ctypes.c_int
    L.rcpsp_server_cancel.argtypes = [vp, ctypes.c_int64]
    L.rcpsp_server_cancel.restype = ctypes.c_int
    L.rcpsp_server_release.argtypes = [vp, ctypes.c_int64]
    L.rcpsp_server_release.restype = ctypes.c_int
    L.rcpsp_server_drain.argtypes = [vp, ctypes.c_int64]
    L.rcpsp_server_drain.restype = ctypes.c_int
    L.rcpsp_server_take_finished.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32, ctypes.POINTER(i32)]
    L.rcpsp_server_take_finished.restype = ctypes.c_int
    L.rcpsp_server_get_stats.argtypes = [vp, ctypes.POINTER(rcpsp_server_stats)]
    L.rcpsp_server_get_stats.restype = ctypes.c_int
    L.rcpsp_server_now_ns.argtypes = []
    L.rcpsp_server_now_ns.restype = ctypes.c_int64
    L.rcpsp_server_destroy.argtypes = [vp]
    L.rcpsp_server_destroy.restype = None
    L.rcpsp_last_error.argtypes = []
    L.rcpsp_last_error.restype = ctypes.c_char_p
    L.rcpsp_version.argtypes = []
    L.rcpsp_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int) -> None:
    if status != 0:
        raise RcpspError(status, lib().rcpsp_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a: Optional[np.ndarray], ct=ctypes.c_int32):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream)) or None


def potential_moves(n: int, swap_range: int) -> int:
    return lib().rcpsp_potential_moves(n, swap_range)


class Instance:
    """A project instance on the current device (rcpsp_create_instance)."""

    def __init__(self, inst, eval: int = EVAL_AUTO):
        L = lib()
        self.n, self.m = inst.n, inst.m
        d, R, r = _i32(inst.duration), _i32(inst.capacity), _i32(inst.request)
        so = _i32(inst.succ_off)
        s = _i32(inst.succ_flat if inst.n_arcs else [0])
        h = ctypes.c_void_p()
        _check(L.rcpsp_create_instance(inst.n, inst.m, _ptr(d), _ptr(R), _ptr(r), _ptr(so), _ptr(s), eval,
                                       ctypes.byref(h)))
        self.h = h

    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.rcpsp_destroy_instance(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    @property
    def info(self) -> dict:
        out = rcpsp_info()
        _check(lib().rcpsp_instance_info(self.h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in rcpsp_info._fields_}

    def evaluate_neighbourhood(self, order: Sequence[int], swap_range: int, tabu: Optional[np.ndarray] = None,
                               aspiration: int = INT32_MAX, stream=None, noalloc: bool = False):
        """Host arrays in and out: returns (makespan[P] with -1 for infeasible
        moves, dict(u, v, makespan, n_feasible)).  noalloc: through
        rcpsp_evaluate_neighbourhood_noalloc (no device allocation)."""
        P = potential_moves(self.n, swap_range)
        mk = np.zeros(max(P, 1), dtype=np.int32)
        best = rcpsp_move()
        npot = ctypes.c_int32()
        tb = None
        if tabu is not None:
            tb = np.ascontiguousarray(np.asarray(tabu, dtype=np.uint8).reshape(self.n * self.n))
        fn = lib().rcpsp_evaluate_neighbourhood_noalloc if noalloc else lib().rcpsp_evaluate_neighbourhood
        order_a = _i32(order)
        _check(fn(self.h, _ptr(order_a), swap_range, tb.ctypes.data if tb is not None else None, aspiration,
                  _ptr(mk), mk.size, ctypes.byref(npot), ctypes.byref(best), _stream_ptr(stream)))
        return mk[:P], dict(u=best.u, v=best.v, makespan=best.makespan, n_feasible=best.n_feasible)

    def evaluate_neighbourhood_device(self, order, swap_range: int, makespan, best, tabu=None,
                                      aspiration: int = INT32_MAX, stream=None) -> None:
        """Device tensors (torch, int32 / uint8): order[N], makespan[P],
        best[4] = (u, v, C_max, n_feasible); asynchronous on `stream`."""
        _check(lib().rcpsp_evaluate_neighbourhood_device(
            self.h, order.data_ptr(), swap_range, tabu.data_ptr() if tabu is not None else None, aspiration,
            makespan.data_ptr() if makespan is not None else None, best.data_ptr(), _stream_ptr(stream)))


def search_params(swap_range: int, tabu_len: int, iterations: int, searches: int = 1, elite: int = 0,
                  phi_max: int = 3, phi_steps: int = 20, threads: int = 0, profile_len: int = 0,
                  record_trajectory: bool = True, count_work: bool = False, full_decode: bool = False,
                  eval: int = EVAL_AUTO, seed: int = 1, lanes: int = 0, fbi: bool = False, exchange_every: int = 0,
                  time_budget_us: int = 0, lane_profile: int = 0) -> rcpsp_search_params:
    return rcpsp_search_params(swap_range, tabu_len, iterations, searches, elite, phi_max, phi_steps, threads,
                               profile_len, int(record_trajectory), int(count_work), int(full_decode), eval, lanes,
                               seed, int(fbi), exchange_every, time_budget_us, lane_profile)


def autotune(instance: "Instance", params: rcpsp_search_params, trial_iterations: int = 10, stream=None):
    """rcpsp_autotune: returns (params with eval/threads/profile_len chosen, tuning dict)."""
    out = rcpsp_search_params()
    info = rcpsp_tuning()
    _check(lib().rcpsp_autotune(instance.h, ctypes.byref(params), trial_iterations, _stream_ptr(stream),
                                ctypes.byref(out), ctypes.byref(info)))
    return out, {k: getattr(info, k) for k, _ in rcpsp_tuning._fields_}


class SearchPlan:
    """rcpsp_search_create / _run / _results / _destroy."""

    def __init__(self, instance: Instance, params: rcpsp_search_params, stream=None):
        self.instance = instance
        self.params = params
        h = ctypes.c_void_p()
        _check(lib().rcpsp_search_create(instance.h, ctypes.byref(params), _stream_ptr(stream), ctypes.byref(h)))
        self.h = h

    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.rcpsp_search_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    @property
    def config(self) -> dict:
        out = rcpsp_search_config()
        _check(lib().rcpsp_search_get_config(self.h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in rcpsp_search_config._fields_}

    def run(self, stream=None) -> None:
        _check(lib().rcpsp_search_run(self.h, _stream_ptr(stream)))

    def run_timed(self, stream=None) -> dict:
        """Eager run with HIP events around every launch: device milliseconds
        of the iteration kernels, the exchange rounds and the whole run."""
        it, rd, tot = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().rcpsp_search_run_timed(self.h, _stream_ptr(stream), ctypes.byref(it), ctypes.byref(rd),
                                            ctypes.byref(tot)))
        return dict(iteration_ms=it.value, round_ms=rd.value, total_ms=tot.value)

    def results(self, stream=None, orders: bool = True, trajectory: bool = True) -> dict:
        p = self.params
        B, N, F = p.searches, self.instance.n, p.elite
        out = dict(best_makespan=np.zeros(B, np.int32), iterations_done=np.zeros(B, np.int32),
                   evaluations=np.zeros(B, np.int64),
                   best_order=np.zeros((B, N), np.int32) if orders else None,
                   trajectory=np.zeros((B, p.iterations, 4), np.int32) if (trajectory and p.record_trajectory) else None,
                   elite_makespan=np.zeros(max(F, 1), np.int32),
                   elite_order=np.zeros((max(F, 1), N), np.int32) if orders else None)
        res = rcpsp_search_result(*[out[k].ctypes.data if out[k] is not None else None for k in
                                    ("best_makespan", "best_order", "iterations_done", "evaluations", "trajectory",
                                     "elite_makespan", "elite_order")])
        _check(lib().rcpsp_search_results(self.h, ctypes.byref(res), _stream_ptr(stream)))
        out["elite_makespan"] = out["elite_makespan"][:F]
        if out["elite_order"] is not None:
            out["elite_order"] = out["elite_order"][:F]
        out["global_best"] = res.global_best
        out["total_evaluations"] = res.total_evaluations
        out["overflow_decodes"] = res.overflow_decodes
        out["total_work"] = res.total_work
        out["total_cells"] = res.total_cells
        return out


def _results(fn, handle_args, params, n, stream, orders=True, trajectory=True, sync=True) -> dict:
    p = params
    B, N, F = p.searches, n, p.elite
    out = dict(best_makespan=np.zeros(B, np.int32), iterations_done=np.zeros(B, np.int32),
               evaluations=np.zeros(B, np.int64),
               best_order=np.zeros((B, N), np.int32) if orders else None,
               trajectory=np.zeros((B, p.iterations, 4), np.int32) if (trajectory and p.record_trajectory) else None,
               elite_makespan=np.zeros(max(F, 1), np.int32),
               elite_order=np.zeros((max(F, 1), N), np.int32) if orders else None)
    res = rcpsp_search_result(*[out[k].ctypes.data if out[k] is not None else None for k in
                                ("best_makespan", "best_order", "iterations_done", "evaluations", "trajectory",
                                 "elite_makespan", "elite_order")])
    if sync:
        _check(fn(*handle_args, ctypes.byref(res), _stream_ptr(stream)))
    else:
        _check(fn(*handle_args, ctypes.byref(res)))
    out["elite_makespan"] = out["elite_makespan"][:F]
    if out["elite_order"] is not None:
        out["elite_order"] = out["elite_order"][:F]
    out["global_best"] = res.global_best
    out["total_evaluations"] = res.total_evaluations
    out["overflow_decodes"] = res.overflow_decodes
    out["total_work"] = res.total_work
    out["total_cells"] = res.total_cells
    return out


def batch_autotune(instances: Sequence["Instance"], params, trial_iterations: int = 5, sample: int = 64,
                   stream=None):
    """rcpsp_batch_autotune: returns (params list with eval/threads chosen, tuning dict)."""
    if not isinstance(params, (list, tuple)):
        params = [params] * len(instances)
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i.h.value for i in instances])
    ps = (rcpsp_search_params * n)(*params)
    out = (rcpsp_search_params * n)()
    info = rcpsp_batch_tuning()
    _check(lib().rcpsp_batch_autotune(hs, n, ps, trial_iterations, sample, _stream_ptr(stream), out,
                                      ctypes.byref(info)))
    g = info.groups
    d = {"groups": g, "trials": info.trials}
    for k in ("group_n", "group_m", "group_members", "group_eval", "group_threads", "group_lanes",
              "group_evals_per_s", "group_register"):
        d[k] = list(getattr(info, k))[:min(g, 8)]
    res = []
    for i in range(n):
        q = rcpsp_search_params()
        ctypes.memmove(ctypes.byref(q), ctypes.byref(out[i]), ctypes.sizeof(q))
        res.append(q)
    return res, d


class Batch:
    """rcpsp_batch_create / _run / _results / _destroy: many instances, each
    with its own search, in persistent launches."""

    def __init__(self, instances: Sequence[Instance], params, stream=None):
        if not isinstance(params, (list, tuple)):
            params = [params] * len(instances)
        self.instances = list(instances)
        self.params = list(params)
        hs = (ctypes.c_void_p * len(instances))(*[i.h.value for i in instances])
        ps = (rcpsp_search_params * len(instances))(*params)
        h = ctypes.c_void_p()
        _check(lib().rcpsp_batch_create(hs, len(instances), ps, _stream_ptr(stream), ctypes.byref(h)))
        self.h = h

    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.rcpsp_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    @property
    def info(self) -> dict:
        out = rcpsp_batch_info()
        _check(lib().rcpsp_batch_get_info(self.h, ctypes.byref(out)))
        d = {"instances": out.instances, "classes": out.classes}
        for k in ("class_eval", "class_threads", "class_instances", "class_workgroups", "class_lds_bytes"):
            d[k] = list(getattr(out, k))[:out.classes]
        return d

    def run(self, stream=None) -> None:
        _check(lib().rcpsp_batch_run(self.h, _stream_ptr(stream)))

    def run_timed(self, stream=None) -> float:
        ms = ctypes.c_double()
        _check(lib().rcpsp_batch_run_timed(self.h, _stream_ptr(stream), ctypes.byref(ms)))
        return ms.value

    def results(self, index: int, stream=None, orders: bool = True, trajectory: bool = True) -> dict:
        return _results(lib().rcpsp_batch_results, (self.h, index), self.params[index], self.instances[index].n,
                        stream, orders, trajectory)


def tabu_search_batch(instances: Sequence[Instance], params, stream=None, orders: bool = True,
                      trajectory: bool = True) -> list:
    """rcpsp_tabu_search_batch: one batch created, run, read and destroyed;
    returns one results dict per instance (as SearchPlan.results)."""
    if not isinstance(params, (list, tuple)):
        params = [params] * len(instances)
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i.h.value for i in instances])
    ps = (rcpsp_search_params * n)(*params)
    outs, ress = [], (rcpsp_search_result * n)()
    for i, p in enumerate(params):
        B, N, F = p.searches, instances[i].n, p.elite
        o = dict(best_makespan=np.zeros(B, np.int32), iterations_done=np.zeros(B, np.int32),
                 evaluations=np.zeros(B, np.int64), best_order=np.zeros((B, N), np.int32) if orders else None,
                 trajectory=np.zeros((B, p.iterations, 4), np.int32) if (trajectory and p.record_trajectory) else None,
                 elite_makespan=np.zeros(max(F, 1), np.int32),
                 elite_order=np.zeros((max(F, 1), N), np.int32) if orders else None)
        ress[i] = rcpsp_search_result(*[o[k].ctypes.data if o[k] is not None else None for k in
                                        ("best_makespan", "best_order", "iterations_done", "evaluations",
                                         "trajectory", "elite_makespan", "elite_order")])
        outs.append(o)
    _check(lib().rcpsp_tabu_search_batch(hs, n, ps, ress, _stream_ptr(stream)))
    for i, o in enumerate(outs):
        F = params[i].elite
        o["elite_makespan"] = o["elite_makespan"][:F]
        if o["elite_order"] is not None:
            o["elite_order"] = o["elite_order"][:F]
        o["global_best"] = ress[i].global_best
        o["total_evaluations"] = ress[i].total_evaluations
        o["overflow_decodes"] = ress[i].overflow_decodes
        o["total_work"] = ress[i].total_work
        o["total_cells"] = ress[i].total_cells
    return outs


class Server:
    """rcpsp_server_*: requests admitted as they arrive, state resident on the
    device, advanced in time slices by a host thread of the library."""

    def __init__(self, max_active: int = 256, slice_us: int = 2000, arena_bytes: int = 2 << 30):
        prm = rcpsp_server_params(max_active, slice_us, arena_bytes)
        h = ctypes.c_void_p()
        _check(lib().rcpsp_server_create(ctypes.byref(prm), ctypes.byref(h)))
        self.h = h
        self._params = {}
        self._inst = {}

    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.rcpsp_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    @staticmethod
    def now_ns() -> int:
        return lib().rcpsp_server_now_ns()

    def submit(self, instance: Instance, params: rcpsp_search_params, budget_us: int = 0) -> int:
        t = ctypes.c_int64()
        _check(lib().rcpsp_server_submit(self.h, instance.h, ctypes.byref(params), budget_us, ctypes.byref(t)))
        self._params[t.value] = params
        self._inst[t.value] = instance
        return t.value

    def poll(self, ticket: int) -> dict:
        st = rcpsp_request_status()
        _check(lib().rcpsp_server_poll(self.h, ticket, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in rcpsp_request_status._fields_}

    def results(self, ticket: int, orders: bool = True, trajectory: bool = True) -> dict:
        return _results(lib().rcpsp_server_results, (self.h, ticket), self._params[ticket],
                        self._inst[ticket].n, None, orders, trajectory, sync=False)

    def cancel(self, ticket: int) -> None:
        _check(lib().rcpsp_server_cancel(self.h, ticket))

    def release(self, ticket: int) -> None:
        _check(lib().rcpsp_server_release(self.h, ticket))
        self._params.pop(ticket, None)
        self._inst.pop(ticket, None)

    def take_finished(self, cap: int = 4096) -> list:
        buf = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        _check(lib().rcpsp_server_take_finished(self.h, buf, cap, ctypes.byref(n)))
        return list(buf[:n.value])

    def drain(self, timeout_ms: int = 0) -> None:
        _check(lib().rcpsp_server_drain(self.h, timeout_ms))

    @property
    def stats(self) -> dict:
        st = rcpsp_server_stats()
        _check(lib().rcpsp_server_get_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in rcpsp_server_stats._fields_}


def tabu_search(instance: Instance, stream=None, **kw) -> dict:
    plan = SearchPlan(instance, search_params(**kw), stream)
    try:
        plan.run(stream)
        return plan.results(stream)
    finally:
        plan.close()


def tabu_search_hosted(instance: Instance, stream=None, **kw) -> dict:
    """rcpsp_tabu_search_hosted: the same independent searches driven by the
    host, one device neighbourhood evaluation per iteration."""
    p = search_params(**kw)
    return _results(lib().rcpsp_tabu_search_hosted, (instance.h, ctypes.byref(p)), p, instance.n, stream)


def tabu_search_reselect(instance: Instance, period: int, probe: int, stream=None, **kw):
    """rcpsp_tabu_search_reselect: the searches of rcpsp_tabu_search with the
    decoder re-chosen by timing at the start of every period.  Returns
    (results, segments), segments a list of dicts in run order."""
    p = search_params(**kw)
    cap = 3 * (p.iterations // max(period, 1) + 1)   # two probes and a chosen run per period
    log = (rcpsp_decoder_segment * cap)()
    n = ctypes.c_int32(0)
    fn = lambda res: lib().rcpsp_tabu_search_reselect(instance.h, ctypes.byref(p), period, probe, res, log, cap,
                                                      ctypes.byref(n), _stream_ptr(stream))
    out = _results(fn, (), p, instance.n, stream, sync=False)
    segs = [{k: getattr(log[i], k) for k, _ in rcpsp_decoder_segment._fields_} for i in range(n.value)]
    return out, segs


def version() -> str:
    return lib().rcpsp_version().decode()
