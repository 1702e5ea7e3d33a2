"""PyTorch plumbing around the C ABI: device memory and streams only.

``simulate`` allocates the workspace and outputs as torch CUDA (HIP) tensors,
runs ``fpt_simulate`` on the current stream and reads the histograms back.
No arithmetic of the method happens here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the fpt library runs on an MI355X (gfx950)")
    return torch


def _aligned_buffer(torch, nbytes: int, device):
    """uint8 device tensor with a 256-byte aligned view of nbytes."""
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw.data_ptr() + off


@dataclasses.dataclass
class SimResult:
    steps: List[Optional["object"]]   # torch int64 tensors (device) or None per set
    hist: "object"                    # torch uint64-as-int64 tensor, all sets
    counts: List[np.ndarray]          # per-set histogram (host)
    moments: List[Dict]               # per-set moments (host)
    stats: Dict


class Plan:
    """An fpt_plan_t with its torch-allocated workspace (reusable)."""

    def __init__(self, sets: Sequence[Dict], precision="fp64", tuning: Optional[Dict] = None,
                 device=None):
        torch = _torch()
        self.sets = [dict(s) for s in sets]
        self.precision = precision
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.handle = _lib.fpt_plan(self.sets, precision, tuning)
        self.ws_bytes = _lib.fpt_plan_workspace(self.handle)
        self._ws_raw, self.ws_ptr = _aligned_buffer(torch, self.ws_bytes, self.device)
        self.n_bins_total = sum(int(s["n_bins"]) for s in self.sets)

    def run(self, record_steps: bool = True, stream=None) -> SimResult:
        torch = _torch()
        current = torch.cuda.current_stream(self.device)
        stream = stream or current
        steps = []
        ptrs = []
        for s in self.sets:
            if record_steps and int(s["n_replicas"]) > 0:
                t = torch.empty(int(s["n_replicas"]), dtype=torch.int64, device=self.device)
                steps.append(t)
                ptrs.append(t.data_ptr())
            else:
                steps.append(None)
                ptrs.append(0)
        hist = torch.empty(max(self.n_bins_total, 1), dtype=torch.int64, device=self.device)
        if stream != current:
            # the outputs (and the workspace) come from the caching allocator
            # on the current stream: order the launch after whatever used that
            # memory before, and keep it from being reused before the launch
            # on `stream` is done
            stream.wait_stream(current)
            for t in [*(t for t in steps if t is not None), hist, self._ws_raw]:
                t.record_stream(stream)
        _lib.fpt_simulate(self.handle, self.ws_ptr, ptrs, hist.data_ptr(), stream.cuda_stream)
        counts, moments = _lib.fpt_histogram_all(self.handle,
                                                 [int(s["n_bins"]) for s in self.sets])
        return SimResult(steps, hist, counts, moments, _lib.fpt_plan_stats(self.handle))

    def close(self):
        if self.handle:
            _lib.fpt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """An fpt_server_t (continuous batching) with its torch-allocated device
    pool and its own stream: ``submit`` queues a job (a dict with the fields
    of ``fpt_params``) and returns its id, ``poll`` returns None while it runs,
    else (counts, moments, latency_s)."""

    def __init__(self, precision="fp32c", model: int = 0, tuning: Optional[Dict] = None,
                 pool_bytes: int = 1 << 30, device=None, scheme: int = 0):
        torch = _torch()
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self._pool_raw, self.pool_ptr = _aligned_buffer(torch, pool_bytes, self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        # the pool was allocated on the current stream; the server writes it
        # on its own stream from creation on
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._pool_raw.record_stream(self.stream)
        self.n_bins: Dict[int, int] = {}
        self.handle = _lib.fpt_server_create(self.pool_ptr, pool_bytes, precision, model,
                                             tuning, self.stream.cuda_stream, scheme)

    def submit(self, params: Dict) -> int:
        job = _lib.fpt_submit(self.handle, params)
        self.n_bins[job] = int(params["n_bins"])
        return job

    def poll(self, job: int):
        return _lib.fpt_poll(self.handle, job, self.n_bins[job])

    def wait(self, job: int, timeout_s: float = 600.0, interval_s: float = 0.005):
        """Poll until the job is done; raises TimeoutError after timeout_s."""
        import time

        t0 = time.perf_counter()
        while True:
            r = self.poll(job)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"job {job} not done after {timeout_s} s")
            time.sleep(interval_s)

    def stats(self) -> Dict:
        return _lib.fpt_server_stats_get(self.handle)

    def close(self):
        if self.handle:
            _lib.fpt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(sets, precision="fp64", tuning: Optional[Dict] = None,
             record_steps: bool = True) -> SimResult:
    """Run every replica of ``sets`` (a dict or a list of dicts with the fields of
    ``fpt_params``) and return escape steps, histograms, moments and stats."""
    if isinstance(sets, dict):
        sets = [sets]
    plan = Plan(sets, precision, tuning)
    try:
        return plan.run(record_steps=record_steps)
    finally:
        plan.close()


def rng_words(seed: int, replica0: int, n_rep: int, block0: int, n_blk: int) -> np.ndarray:
    torch = _torch()
    out = torch.empty(max(n_rep * n_blk * 4, 1), dtype=torch.int32, device="cuda")
    _lib.fpt_rng_words(seed, replica0, n_rep, block0, n_blk, out.data_ptr(),
                       torch.cuda.current_stream().cuda_stream)
    return out[: n_rep * n_blk * 4].cpu().numpy().view(np.uint32).reshape(n_rep, n_blk, 4)


def mt_words(seed: int, replica0: int, n_rep: int, block0: int, n_blk: int) -> np.ndarray:
    """MT19937 words of the FPT_RNG_MT19937 mode, shaped (n_rep, n_blk, 4)."""
    torch = _torch()
    out = torch.empty(max(n_rep * n_blk * 4, 1), dtype=torch.int32, device="cuda")
    _lib.fpt_mt_words(seed, replica0, n_rep, block0, n_blk, out.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
    return out[: n_rep * n_blk * 4].cpu().numpy().view(np.uint32).reshape(n_rep, n_blk, 4)


def normals(seed: int, replica0: int, n_rep: int, block0: int, n_blk: int,
            precision="fp64") -> np.ndarray:
    torch = _torch()
    dt = torch.float64 if _lib.precision_code(precision) == _lib.FPT_FP64 else torch.float32
    out = torch.empty(max(n_rep * n_blk * 4, 1), dtype=dt, device="cuda")
    _lib.fpt_normals(seed, replica0, n_rep, block0, n_blk, precision, out.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
    return out[: n_rep * n_blk * 4].cpu().numpy().reshape(n_rep, n_blk, 4)


def trajectory(params: Dict, replica: int, n_steps: int, precision="fp64"):
    torch = _torch()
    phi = torch.empty(max(n_steps, 1), dtype=torch.float64, device="cuda")
    v = torch.empty(max(n_steps, 1), dtype=torch.float64, device="cuda")
    _lib.fpt_trajectory(params, replica, n_steps, precision, phi.data_ptr(), v.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    return phi[:n_steps].cpu().numpy(), v[:n_steps].cpu().numpy()


def escape_time(steps, dt: float):
    """k*dt in FP64 (Algorithm 1 records k*h); censored (-1) map to -1."""
    k = np.asarray(steps, dtype=np.int64)
    return np.where(k > 0, k.astype(np.float64) * dt, -1.0)


def switching_bias(steps, gamma0: float, ramp: float, dt: float):
    """gamma_k = gamma0 + ramp*dt*k in FP64 (Algorithm 3 records the bias at
    the crossing); censored replicas map to NaN."""
    k = np.asarray(steps, dtype=np.int64)
    return np.where(k > 0, gamma0 + (ramp * dt) * k.astype(np.float64), math.nan)
