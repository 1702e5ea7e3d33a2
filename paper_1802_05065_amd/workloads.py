"""Seeded synthetic workloads (parameter sets and arrival traces).

This module only builds inputs: parameter dictionaries of the five workloads
(plain fixed-bias escape, switching-current ramp, uneven overdamped loads,
batched sets, Poisson serving trace) and the random draws that define the
batched and serving mixes (numpy PCG64).  It holds none of the method's
arithmetic and is shared by the tests (oracle side) and the GPU side.

Field names follow ``fpt_params`` of ``include/fpt.h``; NaN for phi0 / v0 /
threshold selects the paper's defaults (arcsin(gamma0), 0, pi - phi0; the
overdamped model starts at arcsin(gamma0 / V0), the well of its potential).
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

UNDERDAMPED = 0
OVERDAMPED = 1


def base_params(**kw) -> Dict:
    p = dict(
        model=UNDERDAMPED, alpha=0.1, T=0.02, V0=1.0, gamma0=0.0, ramp=0.0, dt=0.01,
        phi0=math.nan, v0=math.nan, threshold=math.nan, max_steps=100000, seed=1,
        n_replicas=1024, n_bins=64, hist_k_max=0, scheme=0, rng=0,
    )
    p.update(kw)
    return p


def plain_escape(n_replicas: int = 1024, seed: int = 1) -> Dict:
    """Fixed bias 0.95, underdamped: alpha 0.1, T 0.02, dt 0.01, phi0 =
    arcsin(0.95), v0 0, escape at phi0 + 2 pi, cap 1e5 steps, 64 bins."""
    phi0 = math.asin(0.95)
    return base_params(
        model=UNDERDAMPED, alpha=0.1, T=0.02, gamma0=0.95, ramp=0.0, dt=0.01,
        phi0=phi0, v0=0.0, threshold=phi0 + 2.0 * math.pi, max_steps=100000,
        seed=seed, n_replicas=n_replicas, n_bins=64, hist_k_max=100000,
    )


def switching_ramp(n_replicas: int = 2 ** 20, seed: int = 2) -> Dict:
    """Switching-current distribution: alpha 0.05, T 0.002, gamma(t) = 1e-6 t
    from 0, dt 0.05 (5e-8 per step), phi0 = v0 = 0, threshold 2 pi, 256 bins
    over gamma in [0, 1] (steps [1, 2e7]); cap 20.1e6 steps (gamma 1.005)."""
    return base_params(
        model=UNDERDAMPED, alpha=0.05, T=0.002, gamma0=0.0, ramp=1e-6, dt=0.05,
        phi0=0.0, v0=0.0, threshold=2.0 * math.pi, max_steps=20_100_000,
        seed=seed, n_replicas=n_replicas, n_bins=256, hist_k_max=20_000_000,
    )


def uneven_overdamped(n_replicas: int = 2 ** 22, seed: int = 3) -> Dict:
    """Overdamped washboard, gamma 0.8, T 0.05, dt 0.01, phi0 = arcsin(0.8),
    threshold phi0 + 2 pi, cap 1e7 steps; exponential-tailed escape times.
    256 bins over steps [1, 1e6]."""
    phi0 = math.asin(0.8)
    return base_params(
        model=OVERDAMPED, alpha=0.0, T=0.05, gamma0=0.8, ramp=0.0, dt=0.01,
        phi0=phi0, v0=0.0, threshold=phi0 + 2.0 * math.pi, max_steps=10_000_000,
        seed=seed, n_replicas=n_replicas, n_bins=256, hist_k_max=1_000_000,
    )


def _ramp_set(u_alpha, u_T, u_ramp, n_replicas, seed, dt=0.05, n_bins=256,
              ramp_scale=1.0) -> Dict:
    alpha = 10.0 ** (-2.0 + 2.0 * u_alpha)
    T = 1e-3 + 4.9e-2 * u_T
    ramp = 10.0 ** (-7.0 + 3.0 * u_ramp) * ramp_scale
    per_step = ramp * dt
    return base_params(
        model=UNDERDAMPED, alpha=alpha, T=T, gamma0=0.0, ramp=ramp, dt=dt,
        phi0=0.0, v0=0.0, threshold=2.0 * math.pi,
        max_steps=int(math.ceil(1.005 / per_step)), seed=seed,
        n_replicas=int(n_replicas), n_bins=n_bins,
        hist_k_max=int(math.ceil(1.0 / per_step)),
    )


def batched_sets(n_sets: int = 256, seed: int = 4, log2_min: float = 12.0,
                 log2_max: float = 16.0, ramp_scale: float = 1.0) -> List[Dict]:
    """Batched mix: alpha log-uniform [0.01, 1], T uniform [1e-3, 5e-2], ramp
    log-uniform [1e-7, 1e-4] per unit time, replicas log-uniform
    2^12..2^16, dt 0.05, gamma from 0, threshold 2 pi; set i has seed
    1000 + i.  ``ramp_scale`` > 1 multiplies every ramp (shorter runs for
    tests); 1 is the workload as defined."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((n_sets, 4))
    sets = []
    for i in range(n_sets):
        n = round(2.0 ** (log2_min + (log2_max - log2_min) * u[i, 3]))
        sets.append(_ramp_set(u[i, 0], u[i, 1], u[i, 2], n, 1000 + i,
                              ramp_scale=ramp_scale))
    return sets


def serving_trace(rate_per_s: float = 50.0, duration_s: float = 60.0, seed: int = 5,
                  log2_min: float = 10.0, log2_max: float = 18.0,
                  ramp_scale: float = 1.0) -> List[Dict]:
    """Poisson arrivals (exponential gaps, mean 1/rate) over ``duration_s``;
    each job is one ramp set drawn as in the batched mix with replicas
    log-uniform 2^10..2^18.  Returns [{'t': arrival_s, 'params': dict}]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        u = rng.random(4)
        n = round(2.0 ** (log2_min + (log2_max - log2_min) * u[3]))
        jobs.append({"t": t, "params": _ramp_set(u[0], u[1], u[2], n, 5000 + i,
                                                  ramp_scale=ramp_scale)})
        i += 1
    return jobs


def to_oracle_kwargs(p: Dict) -> Dict:
    """The subset of fields the oracle's parameter record takes."""
    keys = ("model", "alpha", "T", "V0", "gamma0", "ramp", "dt", "phi0", "v0",
            "threshold", "max_steps", "seed")
    out = {k: p[k] for k in keys}
    out["scheme"] = p.get("scheme", 0)
    out["rng"] = p.get("rng", 0)
    return out
