"""Pins of the oracle's default escape criterion and of the quantities the
GPU tests read from it, against facts that do not come from the oracle:

* Algorithm 1's preamble starts a replica at rest in the well, phi0 =
  arcsin(gamma), and counts an escape once the phase passes the barrier top,
  pi - phi0.  Both points are checked as the minimum and the maximum of the
  tilted washboard potential, found numerically, never through arcsin.
* A noise-free run from the default start with a velocity kick (underdamped)
  or under a ramp (overdamped, V0 != 1) first passes the default threshold at
  the time an independent DOP853 solve of the ODE gives, up to Euler's O(dt)
  error.
* In Eq. (10) V0 multiplies the bias as well as the sine, so the well stays
  at arcsin(gamma) for any V0; the overdamped model's potential is
  -V0 cos(phi) - gamma phi, whose well is at arcsin(gamma / V0): the noise-free
  chain keeps that point and small deviations decay by 1 - dt V0 cos(phi*)
  per step.
* The replica-step count (escape steps, the cap for a censored replica) equals
  the number of (replica, step) pairs still running, summed over the steps.

CPU only (no GPU marker)."""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import minimize_scalar

NAN = math.nan


def _tilted_extrema(model, g, V0):
    """(well, barrier top) of the model's potential on the period around 0 by
    bounded numerical minimisation: V0 (-cos(phi) - g phi) for Eq. (10),
    -V0 cos(phi) - g phi for the overdamped model."""
    if model == 0:
        U = lambda x: V0 * (-math.cos(x) - g * x)  # noqa: E731
    else:
        U = lambda x: -V0 * math.cos(x) - g * x  # noqa: E731
    well = minimize_scalar(U, bounds=(-math.pi / 2, math.pi / 2), method="bounded",
                           options={"xatol": 1e-12}).x
    top = minimize_scalar(lambda x: -U(x), bounds=(math.pi / 2, 3 * math.pi / 2),
                          method="bounded", options={"xatol": 1e-12}).x
    return well, top


@pytest.mark.parametrize("V0", [1.0, 2.5])
@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("g", [-0.9, -0.3, 0.0, 0.3, 0.5, 0.8, 0.95])
def test_default_start_is_the_well_and_threshold_the_barrier_top(oracle_mod, model, g, V0):
    p = oracle_mod.OracleParams(model=model, alpha=0.1, T=0.01, V0=V0, gamma0=g, dt=0.01,
                                phi0=NAN, v0=NAN, threshold=NAN)
    d = oracle_mod.derived(p)
    well, top = _tilted_extrema(model, g, V0)
    assert d["phi0"] == pytest.approx(well, abs=1e-7)
    assert d["threshold"] == pytest.approx(top, abs=1e-7)
    assert d["v0"] == 0.0
    # and to the last bit against the closed forms (the paper's for Eq. (10))
    s = g if model == 0 else g / V0
    assert d["phi0"] == math.asin(s)
    assert d["threshold"] == math.pi - math.asin(s)
    # an explicit value overrides each default on its own
    d2 = oracle_mod.derived(oracle_mod.OracleParams(model=model, gamma0=g, phi0=0.25,
                                                    v0=-1.5, threshold=9.0))
    assert (d2["phi0"], d2["v0"], d2["threshold"]) == (0.25, -1.5, 9.0)


def _first_crossing(rhs, y0, level, t_max):
    def hit(t, y):
        return y[0] - level

    hit.terminal, hit.direction = True, 1
    sol = solve_ivp(rhs, [0.0, t_max], y0, method="DOP853", rtol=1e-12, atol=1e-12,
                    events=hit)
    assert sol.t_events[0].size == 1
    return float(sol.t_events[0][0])


def test_default_criterion_kicked_underdamped_matches_dop853(oracle_mod):
    # at rest in the well a noise-free replica never moves; a velocity kick of
    # 1.4 carries it over the barrier top (pi - arcsin 0.5) once
    g, alpha, v0 = 0.5, 0.1, 1.4
    t_star = _first_crossing(lambda t, y: [y[1], -alpha * y[1] - math.sin(y[0]) + g],
                             [math.asin(g), v0], math.pi - math.asin(g), 50.0)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        p = oracle_mod.OracleParams(model=0, alpha=alpha, T=0.0, gamma0=g, dt=dt,
                                    phi0=NAN, v0=v0, threshold=NAN, max_steps=10**7)
        k = int(oracle_mod.escape_steps(p, 0, 1)[0])
        assert k > 0
        errs.append(abs(k * dt - t_star))
    assert errs[0] < 2.5 * 0.01
    # first-order convergence of the explicit scheme
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]
    # at rest the replica stays in the well: censored
    p = oracle_mod.OracleParams(model=0, alpha=alpha, T=0.0, gamma0=g, dt=0.01,
                                phi0=NAN, v0=NAN, threshold=NAN, max_steps=20_000)
    assert int(oracle_mod.escape_steps(p, 0, 1)[0]) == -1


def test_default_criterion_overdamped_ramp_matches_dop853(oracle_mod):
    # phi' = gamma0 + ramp t - V0 sin(phi) with V0 = 2: the replica follows
    # the well arcsin(gamma(t) / V0) until gamma passes V0, then runs over the
    # initial barrier top pi - arcsin(gamma0 / V0)
    V0, g0, ramp = 2.0, 0.5, 0.05
    start = math.asin(g0 / V0)
    t_star = _first_crossing(lambda t, y: [g0 + ramp * t - V0 * math.sin(y[0])],
                             [start], math.pi - start, 200.0)
    for dt in (0.01, 0.005, 0.0025):
        p = oracle_mod.OracleParams(model=1, alpha=0.0, T=0.0, V0=V0, gamma0=g0, ramp=ramp,
                                    dt=dt, phi0=NAN, v0=NAN, threshold=NAN, max_steps=10**7)
        k = int(oracle_mod.escape_steps(p, 0, 1)[0])
        assert abs(k * dt - t_star) < 2.0 * dt, (dt, k * dt, t_star)


@pytest.mark.parametrize("V0", [0.5, 1.0, 2.5])
def test_overdamped_well_and_relaxation_scale_with_V0(oracle_mod, V0):
    g, dt = 0.3, 0.01
    star = math.asin(g / V0)
    p = oracle_mod.OracleParams(model=1, alpha=0.0, T=0.0, V0=V0, gamma0=g, dt=dt,
                                phi0=NAN, v0=NAN, threshold=1e9, max_steps=2000)
    phi, _ = oracle_mod.trajectory(p, 0, 2000)
    assert np.abs(phi - star).max() < 1e-12
    # a small displacement decays geometrically by 1 - dt V0 cos(phi*)
    eps = 1e-6
    p = oracle_mod.OracleParams(model=1, alpha=0.0, T=0.0, V0=V0, gamma0=g, dt=dt,
                                phi0=star + eps, v0=NAN, threshold=1e9, max_steps=50)
    phi, _ = oracle_mod.trajectory(p, 0, 50)
    dev = np.concatenate([[eps], phi - star])
    ratio = dev[1:20] / dev[:19]
    assert ratio == pytest.approx(1.0 - dt * V0 * math.cos(star), abs=2e-5)


def test_replica_steps_is_the_survival_sum(oracle_mod):
    # sum over steps k = 1..cap of the replicas still running at step k:
    # an escaped replica runs its k steps, a censored one all cap steps
    cap = 257
    rng = np.random.Generator(np.random.PCG64(8))
    steps = rng.integers(1, cap + 1, size=3000).astype(np.int64)
    steps[rng.random(3000) < 0.2] = -1
    steps[:3] = [1, cap, -1]
    running = sum(int(np.count_nonzero((steps >= k) | (steps == -1))) for k in range(1, cap + 1))
    assert oracle_mod.replica_steps(steps, cap) == running
    # the same identity on a run of the oracle itself with censored replicas
    p = oracle_mod.OracleParams(model=0, alpha=0.1, T=0.02, gamma0=0.95, dt=0.01,
                                phi0=NAN, v0=NAN, threshold=NAN, max_steps=1500, seed=4)
    run = oracle_mod.escape_steps(p, 0, 400)
    assert (run == -1).any() and (run > 0).any()
    running = sum(int(np.count_nonzero((run >= k) | (run == -1))) for k in range(1, 1501))
    assert oracle_mod.replica_steps(run, 1500) == running
