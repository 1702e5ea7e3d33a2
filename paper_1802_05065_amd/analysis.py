"""Applications of the library that reproduce the paper's physics checks.

* Sect. IV.A (Arrhenius plots): mean first-passage time over a range of
  temperatures at fixed bias, and the barrier height recovered from the slope
  of ln<tau> against 1/T (Eq. (13)) or of ln(T <tau>) (the prefactor form of
  Eq. (14), whose slope is the quasipotential estimate of Eq. (15)).
* Sect. IV.B (switching-current distributions): the switching-bias CDF of a
  linear ramp against the adiabatic theory of Fulton and Dunkleberger,
  P(gamma) = 1 - exp(-int_0^gamma Gamma(u) du / (d gamma/dt)), with the
  moderate-damping Kramers rate Gamma.

All integration runs in the library's kernels (one batched plan per sweep);
this module only builds parameter sets and evaluates closed-form theory on
the host.

Both theories assume the continuous-time Langevin equation.  The Euler
schemes sample a slightly different stationary state: linearized at the well
bottom (frequency^2 = V0 sqrt(1 - gamma^2)), Algorithm 1's explicit update
lowers the effective damping by dt frequency^2 and so heats the well, while
the semi-implicit update keeps it at T to O(dt^2).  `scheme_temperature`
gives that stationary temperature from the discrete Lyapunov equation of the
linearized scheme, and the theory can be evaluated with it.
"""

from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import api, workloads


def barrier_height(gamma, V0: float = 1.0):
    """Delta U of the tilted washboard -V0 (cos phi + gamma phi):
    2 V0 [sqrt(1 - gamma^2) - gamma arccos(gamma)]."""
    g = np.asarray(gamma, dtype=np.float64)
    return 2.0 * V0 * (np.sqrt(1.0 - g * g) - g * np.arccos(g))


def kramers_rate(gamma, alpha: float, T: float, V0: float = 1.0):
    """Escape rate over the washboard barrier at moderate damping
    (units: the library's time): (omega_a / 2 pi) (sqrt(alpha^2/4 + omega_b^2)
    - alpha/2) / omega_b exp(-Delta U / T), omega_a = omega_b =
    sqrt(V0) (1 - gamma^2)^(1/4)."""
    g = np.asarray(gamma, dtype=np.float64)
    w = math.sqrt(V0) * (1.0 - g * g) ** 0.25
    lam = np.sqrt(alpha * alpha / 4.0 + w * w) - alpha / 2.0
    return w / (2.0 * math.pi) * (lam / w) * np.exp(-barrier_height(g, V0) / T)


def scheme_temperature(gamma, alpha: float, T: float, dt: float, scheme: int,
                       V0: float = 1.0):
    """Stationary temperature (omega^2 <dphi^2>) of the underdamped Euler
    scheme linearized at the well bottom of bias gamma: 0 explicit
    (Algorithm 1), 1 semi-implicit.  Equals T in the limit dt -> 0."""
    from scipy.linalg import solve_discrete_lyapunov

    g = np.atleast_1d(np.asarray(gamma, dtype=np.float64))
    out = np.empty_like(g)
    for i, gi in enumerate(g):
        w2 = V0 * math.sqrt(max(1.0 - gi * gi, 0.0))
        h = dt
        if scheme == 0:
            A = np.array([[1.0, h], [-h * w2, 1.0 - h * alpha]])
            b = np.array([0.0, 1.0])
        else:
            A = np.array([[1.0 - h * h * w2, h * (1.0 - h * alpha)], [-h * w2, 1.0 - h * alpha]])
            b = np.array([h, 1.0])
        C = solve_discrete_lyapunov(A, 2.0 * alpha * T * h * np.outer(b, b))
        out[i] = w2 * C[0, 0]
    return out if np.ndim(gamma) else float(out[0])


def fulton_dunkleberger_cdf(gamma_grid, alpha: float, T: float, ramp: float,
                            V0: float = 1.0, n_quad: int = 20000,
                            dt: Optional[float] = None, scheme: int = 0):
    """Adiabatic switching-bias CDF for a bias ramped at `ramp` per unit time
    from 0: P(gamma) = 1 - exp(-(1/ramp) int_0^gamma Gamma(u) du).  With `dt`
    the rate at each bias uses the scheme's stationary temperature instead of
    T (see scheme_temperature)."""
    grid = np.asarray(gamma_grid, dtype=np.float64)
    top = float(min(grid.max(), 1.0 - 1e-12))
    u = np.linspace(0.0, top, n_quad)
    if dt is None:
        rate = kramers_rate(u, alpha, T, V0)
    else:
        coarse = np.linspace(0.0, top, 200)
        t_eff = np.interp(u, coarse, scheme_temperature(coarse, alpha, T, dt, scheme, V0))
        rate = np.array([kramers_rate(x, alpha, te, V0) for x, te in zip(u, t_eff)])
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (rate[1:] + rate[:-1]) * np.diff(u))])
    return 1.0 - np.exp(-np.interp(np.minimum(grid, top), u, cum) / ramp)


def barrier_fits(temperatures, tau, se=None) -> Dict:
    """Barrier heights from mean first-passage times over temperatures:
    the slope of ln<tau> against 1/T (the Arrhenius law, Eq. (13)) and the
    slope of ln(T <tau>) against 1/T (the prefactor form of Eq. (14), read
    as the quasipotential estimate of Eq. (15)), each a least-squares line
    weighted by 1 / var(ln tau) when standard errors are given, with the
    slope's standard error."""
    T = np.asarray(temperatures, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    x = 1.0 / T
    w = np.ones_like(tau) if se is None else (tau / np.asarray(se, dtype=np.float64)) ** 2
    out = {}
    for name, y in (("arrhenius", np.log(tau)), ("kramers_form", np.log(T * tau))):
        W = w.sum()
        xm, ym = (w * x).sum() / W, (w * y).sum() / W
        sxx = (w * (x - xm) ** 2).sum()
        slope = (w * (x - xm) * (y - ym)).sum() / sxx
        out[f"delta_U_{name}"] = float(slope)
        # with known variances 1/w of the points, var(slope) = 1 / sxx
        out[f"delta_U_{name}_se"] = float(math.sqrt(1.0 / sxx)) if se is not None else None
    return out


def arrhenius_sweep(gamma: float, alpha: float, temperatures: Sequence[float],
                    n_replicas: int = 4096, dt: float = 0.02, V0: float = 1.0,
                    precision: str = "fp32c", seed: int = 100,
                    max_steps: Optional[int] = None, scheme: int = 0,
                    threshold: str = "period", record_steps: bool = False) -> Dict:
    """Mean first-passage time from the well bottom at each temperature, in
    one batched plan, and the barrier fitted from it (``barrier_fits``), beside
    the same fits of the moderate-damping Kramers times at those
    temperatures.  ``threshold``: "period" escapes at phi0 + 2 pi (the next
    well); "barrier" uses Algorithm 1's own criterion, NaN start and
    threshold (at rest in the well, escape past the barrier top
    pi - arcsin(gamma)).  ``record_steps`` adds every set's escape steps
    (host int64 arrays) as "steps"."""
    phi0 = math.asin(gamma)
    temps = [float(t) for t in temperatures]
    du = float(barrier_height(gamma, V0))
    if threshold == "period":
        start = dict(phi0=phi0, v0=0.0, threshold=phi0 + 2.0 * math.pi)
    elif threshold == "barrier":
        start = dict(phi0=math.nan, v0=math.nan, threshold=math.nan)
    else:
        raise ValueError(f"threshold {threshold!r}: 'period' or 'barrier'")
    sets = []
    for i, T in enumerate(temps):
        tau_est = 1.0 / float(kramers_rate(gamma, alpha, T, V0))
        cap = max_steps or int(min(2 ** 40, 40 * tau_est / dt + 1e5))
        sets.append(workloads.base_params(
            model=workloads.UNDERDAMPED, alpha=alpha, T=T, V0=V0, gamma0=gamma, ramp=0.0,
            dt=dt, max_steps=cap, seed=seed + i, n_replicas=n_replicas, n_bins=64,
            hist_k_max=cap, **start) | {"scheme": scheme})
    res = api.simulate(sets, precision, record_steps=record_steps)
    tau = np.array([m["mean_t"] for m in res.moments])
    se = np.array([m["se_t"] for m in res.moments])
    cens = [int(m["n_censored"]) for m in res.moments]
    steps = [s.cpu().numpy() for s in res.steps] if record_steps else None
    tau_k = [1.0 / float(kramers_rate(gamma, alpha, T, V0)) for T in temps]
    fits = barrier_fits(temps, tau, se)
    theory = barrier_fits(temps, tau_k, np.array(tau_k) * se / tau)
    return {"temperatures": temps, "mean_fpt": tau.tolist(), "se": se.tolist(),
            "censored": cens, "delta_U": du, **fits,
            "kramers_tau": tau_k,
            "theory_delta_U_arrhenius": theory["delta_U_arrhenius"],
            "theory_delta_U_kramers_form": theory["delta_U_kramers_form"],
            "sets": sets, "steps": steps, "stats": res.stats}


def switching_distribution(alpha: float, T: float, ramp: float, n_replicas: int = 30000,
                           dt: float = 0.05, V0: float = 1.0, precision: str = "fp32c",
                           seed: int = 200, n_bins: int = 1024, scheme: int = 0) -> Dict:
    """Switching-bias distribution of a linear ramp from gamma = 0 (the
    switching-current kernel, Algorithm 3) and its adiabatic prediction, at T
    ("theory") and at the scheme's stationary temperature ("theory_scheme")."""
    per_step = ramp * dt
    k1 = int(math.ceil(1.0 / per_step))
    p = workloads.base_params(
        model=workloads.UNDERDAMPED, alpha=alpha, T=T, V0=V0, gamma0=0.0, ramp=ramp, dt=dt,
        phi0=0.0, v0=0.0, threshold=2.0 * math.pi, max_steps=int(math.ceil(1.005 / per_step)),
        seed=seed, n_replicas=n_replicas, n_bins=n_bins, hist_k_max=k1)
    p["scheme"] = scheme
    res = api.simulate(p, precision, record_steps=True)
    steps = res.steps[0].cpu().numpy()
    g = api.switching_bias(steps, 0.0, ramp, dt)
    g = np.sort(g[np.isfinite(g)])
    emp = np.arange(1, g.size + 1) / n_replicas
    theory = fulton_dunkleberger_cdf(g, alpha, T, ramp, V0)
    theory_s = fulton_dunkleberger_cdf(g, alpha, T, ramp, V0, dt=dt, scheme=scheme)
    return {"gamma_sw": g, "cdf": emp, "theory": theory, "theory_scheme": theory_s,
            "max_abs_diff": float(np.max(np.abs(emp - theory))) if g.size else None,
            "max_abs_diff_scheme": float(np.max(np.abs(emp - theory_s))) if g.size else None,
            "mean_gamma_sw": float(g.mean()) if g.size else None,
            "counts": res.counts[0], "stats": res.stats}
