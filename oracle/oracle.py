"""ctypes wrapper of the C oracle (``fpt_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Every function here runs the plain single-threaded
FP64 C code; nothing in this module calls the GPU library.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpt_oracle.c")
_CLI_SRC = os.path.join(_HERE, "fpt_oracle_cli.c")
_LIB = os.path.join(_HERE, "libfpt_oracle.so")
_CLI = os.path.join(_HERE, "fpt_oracle_cli")
_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(force: bool = True) -> None:
    """Compile the oracle library and its CLI with gcc (IEEE double, no FMA
    contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(
            ["gcc", *_CFLAGS, "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        )
        os.replace(_LIB + ".tmp", _LIB)
    if force or not os.path.exists(_CLI):
        subprocess.check_call(
            ["gcc", *_CFLAGS, "-o", _CLI + ".tmp", _CLI_SRC, _SRC, "-lm"]
        )
        os.replace(_CLI + ".tmp", _CLI)


class _CParams(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("rng", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
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
        ("seed", ctypes.c_uint64),
    ]


class _CMoments(ctypes.Structure):
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


@dataclasses.dataclass
class OracleParams:
    """One parameter set.  ``model``: 0 underdamped, 1 overdamped.  NaN for
    phi0 / v0 / threshold selects the paper's defaults (arcsin(gamma0), 0,
    pi - phi0; overdamped: arcsin(gamma0 / V0), the well of its potential)."""

    model: int = 0
    alpha: float = 0.1
    T: float = 0.02
    V0: float = 1.0
    gamma0: float = 0.0
    ramp: float = 0.0
    dt: float = 0.01
    phi0: float = math.nan
    v0: float = math.nan
    threshold: float = math.nan
    max_steps: int = 100000
    seed: int = 1
    scheme: int = 0
    rng: int = 0

    def _c(self) -> _CParams:
        return _CParams(
            int(self.model), int(self.scheme), int(self.rng), 0, float(self.alpha), float(self.T), float(self.V0),
            float(self.gamma0), float(self.ramp), float(self.dt), float(self.phi0),
            float(self.v0), float(self.threshold), int(self.max_steps),
            int(self.seed) & 0xFFFFFFFFFFFFFFFF,
        )


_lib_handle: Optional[ctypes.CDLL] = None


def _lib() -> ctypes.CDLL:
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        f64p = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_CParams)
        lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.oracle_rng_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u32p]
        lib.oracle_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.oracle_derived.argtypes = [pp, f64p, f64p, f64p, f64p, f64p]
        lib.oracle_escape_step.argtypes = [pp, ctypes.c_uint64, f64p, f64p]
        lib.oracle_escape_step.restype = ctypes.c_int64
        lib.oracle_run.argtypes = [pp, ctypes.c_uint64, ctypes.c_uint64, i64p, f64p]
        lib.oracle_trajectory.argtypes = [pp, ctypes.c_uint64, ctypes.c_int64, f64p, f64p]
        lib.oracle_histogram.argtypes = [
            i64p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
            u64p, ctypes.POINTER(_CMoments),
        ]
        lib.oracle_mt19937.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p]
        lib.oracle_replica_steps.argtypes = [i64p, ctypes.c_uint64, ctypes.c_int64]
        lib.oracle_replica_steps.restype = ctypes.c_uint64
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one counter (4 words) and key (2 words)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _lib().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                                _ptr(out, ctypes.c_uint32))
    return out


def rng_words(seed: int, replica: int, block: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    _lib().oracle_rng_words(seed & (2**64 - 1), replica, block, _ptr(out, ctypes.c_uint32))
    return out


def mt19937(seed: int, n: int) -> np.ndarray:
    """First n outputs of MT19937 with the standard 32-bit seeding."""
    out = np.zeros(max(n, 1), dtype=np.uint32)
    _lib().oracle_mt19937(seed & 0xFFFFFFFF, n, _ptr(out, ctypes.c_uint32))
    return out[:n]


def normals(seed: int, replica: int, block: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.float64)
    _lib().oracle_normals(seed & (2**64 - 1), replica, block, _ptr(out, ctypes.c_double))
    return out


def derived(p: OracleParams) -> dict:
    vals = [ctypes.c_double() for _ in range(5)]
    cp = p._c()
    _lib().oracle_derived(ctypes.byref(cp), *[ctypes.byref(v) for v in vals])
    names = ["sigma", "dgamma", "phi0", "v0", "threshold"]
    return {n: v.value for n, v in zip(names, vals)}


def escape_steps(p: OracleParams, first: int, n: int, with_phi: bool = False):
    """Escape steps of replicas first..first+n-1 (int64, -1 = censored)."""
    steps = np.zeros(max(n, 1), dtype=np.int64)
    phi = np.zeros(max(n, 1), dtype=np.float64) if with_phi else None
    cp = p._c()
    _lib().oracle_run(ctypes.byref(cp), first, n, _ptr(steps, ctypes.c_int64),
                      _ptr(phi, ctypes.c_double) if with_phi else None)
    if with_phi:
        return steps[:n], phi[:n]
    return steps[:n]


def trajectory(p: OracleParams, replica: int, n_steps: int):
    phi = np.zeros(n_steps, dtype=np.float64)
    v = np.zeros(n_steps, dtype=np.float64)
    cp = p._c()
    _lib().oracle_trajectory(ctypes.byref(cp), replica, n_steps,
                             _ptr(phi, ctypes.c_double), _ptr(v, ctypes.c_double))
    return phi, v


def histogram(steps: np.ndarray, n_bins: int, k_hist: int, dt: float):
    """(hist uint64[n_bins], moments dict) of an escape-step array."""
    s = np.ascontiguousarray(np.asarray(steps, dtype=np.int64))
    hist = np.zeros(n_bins, dtype=np.uint64)
    m = _CMoments()
    _lib().oracle_histogram(_ptr(s, ctypes.c_int64), s.size, n_bins, k_hist, dt,
                            _ptr(hist, ctypes.c_uint64), ctypes.byref(m))
    mom = {f[0]: getattr(m, f[0]) for f in _CMoments._fields_}
    mom["sum_k2"] = (mom["sum_k2_hi"] << 64) | mom["sum_k2_lo"]
    return hist, mom


def replica_steps(steps: np.ndarray, max_steps: int) -> int:
    s = np.ascontiguousarray(np.asarray(steps, dtype=np.int64))
    return int(_lib().oracle_replica_steps(_ptr(s, ctypes.c_int64), s.size, max_steps))


def run_cli(p: OracleParams, first: int, n: int):
    """Run the oracle CLI as a child process (used to time it on several host
    cores at once).  Returns (replica_steps, n_escaped, seconds, steps)."""
    if not os.path.exists(_CLI):
        build(force=False)
    args = [
        _CLI, str(p.model), repr(p.alpha), repr(p.T), repr(p.V0), repr(p.gamma0),
        repr(p.ramp), repr(p.dt), repr(p.phi0), repr(p.v0), repr(p.threshold),
        str(int(p.max_steps)), str(int(p.seed)), str(first), str(n),
    ]
    out = subprocess.check_output(args, text=True)
    lines = out.split("\n")
    head = lines[0].split()
    steps = np.array([int(x) for x in lines[1:1 + n]], dtype=np.int64)
    return int(head[2]), int(head[3]), float(head[4]), steps
