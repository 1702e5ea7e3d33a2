"""ctypes binding of ``libfpt.so`` (the C ABI of ``include/fpt.h``).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of the library.  Importing this module does not touch the GPU; the
first call loads the library and raises if it has not been built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpt.so")

FPT_OK = 0
FPT_PENDING = 1
FPT_E_INVAL = -1
FPT_E_NOMEM = -2
FPT_E_DEVICE = -3
FPT_E_BUSY = -4
FPT_E_NOTFOUND = -5
FPT_E_STATE = -6

FPT_UNDERDAMPED = 0
FPT_OVERDAMPED = 1
FPT_EXPLICIT = 0
FPT_SEMI_IMPLICIT = 1
FPT_RNG_PHILOX = 0
FPT_RNG_MT19937 = 1
FPT_FP64 = 0
FPT_FP32C = 1
FPT_SCHED_REFILL = 0
FPT_SCHED_ONE_PER_LANE = 1
FPT_MAX_BINS = 4096

PRECISIONS = {"fp64": FPT_FP64, "fp32c": FPT_FP32C}


def precision_code(p) -> int:
    """'fp64' / 'fp32c' or the integer code itself (passed through unchecked:
    the library validates it)."""
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class FptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fpt status {status}: {message}")
        self.status = status
        self.message = message


class FptParams(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("rng", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("T", ctypes.c_double),
        ("V0", ctypes.c_double),
        ("gamma0", ctypes.c_double),
        ("ramp", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("phi0", ctypes.c_double),
        ("v0", ctypes.c_double),
        ("threshold", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("n_replicas", ctypes.c_int64),
        ("hist_k_max", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
    ]


class FptTuning(ctypes.Structure):
    _fields_ = [
        ("schedule", ctypes.c_int32),
        ("replicas_per_lane", ctypes.c_int32),
        ("waves_per_simd", ctypes.c_int32),
        ("steps_per_launch", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("no_compaction", ctypes.c_int32),
        ("no_regroup", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class FptMoments(ctypes.Structure):
    _fields_ = [
        ("n_escaped", ctypes.c_uint64),
        ("n_censored", ctypes.c_uint64),
        ("n_overflow", ctypes.c_uint64),
        ("sum_k", ctypes.c_uint64),
        ("sum_k2_lo", ctypes.c_uint64),
        ("sum_k2_hi", ctypes.c_uint64),
        ("mean_t", ctypes.c_double),
        ("se_t", ctypes.c_double),
    ]


class FptRunStats(ctypes.Structure):
    _fields_ = [
        ("replica_steps", ctypes.c_uint64),
        ("lane_steps", ctypes.c_uint64),
        ("n_launches", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double),
        ("wall_ms", ctypes.c_double),
        ("tuning", FptTuning),
        ("n_compactions", ctypes.c_int64),
        ("n_regroups", ctypes.c_int64),
        ("extra_passes", ctypes.c_uint64),
    ]


class FptServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("finished", ctypes.c_uint64),
        ("queued", ctypes.c_uint64),
        ("running", ctypes.c_uint64),
        ("replica_steps", ctypes.c_uint64),
        ("n_launches", ctypes.c_int64),
        ("busy_s", ctypes.c_double),
        ("n_compactions", ctypes.c_int64),
        ("n_regroups", ctypes.c_int64),
    ]


# (name, restype, argtypes) of every entry point of include/fpt.h
_VP = ctypes.c_void_p
SIGNATURES = [
    ("fpt_plan", ctypes.c_int, [ctypes.POINTER(FptParams), ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(FptTuning), ctypes.POINTER(_VP)]),
    ("fpt_plan_workspace", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    ("fpt_simulate", ctypes.c_int, [_VP, _VP, ctypes.POINTER(_VP), _VP, _VP]),
    ("fpt_simulate_noalloc", ctypes.c_int, [_VP, ctypes.POINTER(_VP), _VP, _VP]),
    ("fpt_histogram", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(FptMoments)]),
    ("fpt_histogram_all", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(FptMoments)]),
    ("fpt_plan_stats", ctypes.c_int, [_VP, ctypes.POINTER(FptRunStats)]),
    ("fpt_plan_destroy", None, [_VP]),
    ("fpt_server_create", ctypes.c_int, [_VP, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(FptTuning), _VP,
                                         ctypes.POINTER(_VP)]),
    ("fpt_submit", ctypes.c_int, [_VP, ctypes.POINTER(FptParams),
                                  ctypes.POINTER(ctypes.c_uint64)]),
    ("fpt_poll", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(FptMoments), ctypes.POINTER(ctypes.c_double)]),
    ("fpt_server_stats_get", ctypes.c_int, [_VP, ctypes.POINTER(FptServerStats)]),
    ("fpt_server_destroy", None, [_VP]),
    ("fpt_rng_words", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_uint64, ctypes.c_int64, _VP, _VP]),
    ("fpt_mt_words", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                    ctypes.c_uint64, ctypes.c_int64, _VP, _VP]),
    ("fpt_normals", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                   ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, _VP, _VP]),
    ("fpt_trajectory", ctypes.c_int, [ctypes.POINTER(FptParams), ctypes.c_uint64,
                                      ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP]),
    ("fpt_last_error", ctypes.c_char_p, []),
    ("fpt_api_version", ctypes.c_int32, []),
]

_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if ``libfpt.so`` has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(python -m paper_1802_05065_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def last_error() -> str:
    msg = lib().fpt_last_error()
    return msg.decode() if msg else ""


def check(status: int, allow=(FPT_OK,)) -> int:
    if status in allow:
        return status
    raise FptError(status, last_error())


def make_params(p: Dict) -> FptParams:
    """fpt_params from a dict with the field names of include/fpt.h."""
    return FptParams(
        int(p["model"]), int(p["n_bins"]), int(p.get("scheme", 0)), int(p.get("rng", 0)),
        float(p["alpha"]), float(p["T"]),
        float(p.get("V0", 1.0)), float(p["gamma0"]), float(p["ramp"]), float(p["dt"]),
        float(p["phi0"]), float(p["v0"]), float(p["threshold"]), int(p["max_steps"]),
        int(p["n_replicas"]), int(p.get("hist_k_max", 0)), int(p["seed"]) & (2**64 - 1),
    )


def make_tuning(t: Optional[Dict]) -> Optional[FptTuning]:
    if t is None:
        return None
    return FptTuning(int(t.get("schedule", 0)), int(t.get("replicas_per_lane", 0)),
                     int(t.get("waves_per_simd", 0)), int(t.get("steps_per_launch", 0)),
                     int(t.get("use_graph", 0)), int(t.get("no_compaction", 0)),
                     int(t.get("no_regroup", 0)))


def moments_dict(m: FptMoments) -> Dict:
    d = {f[0]: getattr(m, f[0]) for f in FptMoments._fields_}
    d["sum_k2"] = (d["sum_k2_hi"] << 64) | d["sum_k2_lo"]
    return d


# ---- same-name wrappers -----------------------------------------------------

def fpt_plan(sets: Sequence[Dict], precision, tuning: Optional[Dict] = None) -> int:
    arr = (FptParams * len(sets))(*[make_params(s) for s in sets])
    t = make_tuning(tuning)
    out = ctypes.c_void_p()
    check(lib().fpt_plan(arr, len(sets), precision_code(precision),
                         ctypes.byref(t) if t is not None else None, ctypes.byref(out)))
    return out.value


def fpt_plan_workspace(plan: int) -> int:
    n = ctypes.c_size_t()
    check(lib().fpt_plan_workspace(plan, ctypes.byref(n)))
    return n.value


def fpt_simulate(plan: int, workspace: int, out_steps: Optional[Sequence[int]],
                 out_hist: Optional[int], stream: Optional[int]) -> None:
    steps_arr = None
    if out_steps is not None:
        steps_arr = (ctypes.c_void_p * len(out_steps))(*[p or None for p in out_steps])
    check(lib().fpt_simulate(plan, workspace, steps_arr, out_hist or None, stream or None))


def fpt_simulate_noalloc(plan: int, out_steps: Optional[Sequence[int]],
                         out_hist: Optional[int], stream: Optional[int]) -> None:
    steps_arr = None
    if out_steps is not None:
        steps_arr = (ctypes.c_void_p * len(out_steps))(*[p or None for p in out_steps])
    check(lib().fpt_simulate_noalloc(plan, steps_arr, out_hist or None, stream or None))


NOALLOC_SCRATCH_BYTES = 48 << 20  # FPT_NOALLOC_SCRATCH_BYTES of include/fpt.h


def fpt_histogram(plan: int, set_index: int, n_bins: int):
    counts = np.zeros(n_bins, dtype=np.uint64)
    m = FptMoments()
    check(lib().fpt_histogram(plan, set_index,
                              counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                              ctypes.byref(m)))
    return counts, moments_dict(m)


def fpt_histogram_all(plan: int, n_bins: Sequence[int]):
    """Every set's counts (list of arrays, plan order) and moments."""
    total = int(sum(n_bins))
    counts = np.zeros(max(total, 1), dtype=np.uint64)
    moms = (FptMoments * max(len(n_bins), 1))()
    check(lib().fpt_histogram_all(plan, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  moms))
    out_c, off = [], 0
    for n in n_bins:
        out_c.append(counts[off:off + int(n)].copy())
        off += int(n)
    return out_c, [moments_dict(moms[i]) for i in range(len(n_bins))]


def fpt_plan_stats(plan: int) -> Dict:
    s = FptRunStats()
    check(lib().fpt_plan_stats(plan, ctypes.byref(s)))
    t = s.tuning
    return dict(replica_steps=s.replica_steps, lane_steps=s.lane_steps,
                n_launches=s.n_launches, kernel_ms=s.kernel_ms, wall_ms=s.wall_ms,
                n_compactions=s.n_compactions, n_regroups=s.n_regroups,
                extra_passes=s.extra_passes,
                tuning=dict(schedule=t.schedule, replicas_per_lane=t.replicas_per_lane,
                            waves_per_simd=t.waves_per_simd,
                            steps_per_launch=t.steps_per_launch, use_graph=t.use_graph,
                            no_compaction=t.no_compaction, no_regroup=t.no_regroup))


def fpt_plan_destroy(plan: int) -> None:
    if plan:
        lib().fpt_plan_destroy(plan)


def fpt_server_create(pool: int, pool_bytes: int, precision, model: int,
                      tuning: Optional[Dict], stream: Optional[int], scheme: int = 0) -> int:
    t = make_tuning(tuning)
    out = ctypes.c_void_p()
    check(lib().fpt_server_create(pool, pool_bytes, precision_code(precision), model, scheme,
                                  ctypes.byref(t) if t is not None else None, stream or None,
                                  ctypes.byref(out)))
    return out.value


def fpt_submit(server: int, params: Dict) -> int:
    p = make_params(params)
    job = ctypes.c_uint64()
    check(lib().fpt_submit(server, ctypes.byref(p), ctypes.byref(job)))
    return job.value


def fpt_poll(server: int, job: int, n_bins: int):
    """None while pending, else (counts, moments, latency_s)."""
    counts = np.zeros(n_bins, dtype=np.uint64)
    m = FptMoments()
    lat = ctypes.c_double()
    st = check(lib().fpt_poll(server, job,
                              counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                              ctypes.byref(m), ctypes.byref(lat)), allow=(FPT_OK, FPT_PENDING))
    if st == FPT_PENDING:
        return None
    return counts, moments_dict(m), lat.value


def fpt_server_stats_get(server: int) -> Dict:
    s = FptServerStats()
    check(lib().fpt_server_stats_get(server, ctypes.byref(s)))
    return {f[0]: getattr(s, f[0]) for f in FptServerStats._fields_}


def fpt_server_destroy(server: int) -> None:
    if server:
        lib().fpt_server_destroy(server)


def fpt_rng_words(seed, replica0, n_rep, block0, n_blk, out_ptr, stream) -> None:
    check(lib().fpt_rng_words(seed & (2**64 - 1), replica0, n_rep, block0, n_blk, out_ptr,
                              stream or None))


def fpt_mt_words(seed, replica0, n_rep, block0, n_blk, out_ptr, stream) -> None:
    check(lib().fpt_mt_words(seed & (2**64 - 1), replica0, n_rep, block0, n_blk, out_ptr,
                             stream or None))


def fpt_normals(seed, replica0, n_rep, block0, n_blk, precision, out_ptr, stream) -> None:
    check(lib().fpt_normals(seed & (2**64 - 1), replica0, n_rep, block0, n_blk,
                            precision_code(precision), out_ptr, stream or None))


def fpt_trajectory(params: Dict, replica: int, n_steps: int, precision, phi_ptr, v_ptr,
                   stream) -> None:
    p = make_params(params)
    check(lib().fpt_trajectory(ctypes.byref(p), replica, n_steps, precision_code(precision),
                               phi_ptr, v_ptr, stream or None))


def fpt_last_error() -> str:
    return last_error()


def fpt_api_version() -> int:
    return int(lib().fpt_api_version())
