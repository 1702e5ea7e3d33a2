"""The paper's physics checks run through the library (GPU): the barrier
height recovered from an Arrhenius sweep (Sect. IV.A), and the switching
distribution of a slow ramp against the adiabatic Fulton-Dunkleberger theory
(Sect. IV.B).  Both compare with closed-form physics, not with the oracle."""

import numpy as np
import pytest

from paper_1802_05065_amd import analysis

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_arrhenius_barrier(precision):
    g, alpha = 0.5, 0.5
    du = float(analysis.barrier_height(g))
    temps = [du / r for r in (4.0, 5.0, 6.0, 7.0)]
    out = analysis.arrhenius_sweep(g, alpha, temps, n_replicas=4096, dt=0.02,
                                   precision=precision)
    print(out["delta_U"], out["delta_U_arrhenius"], out["delta_U_kramers_form"],
          out["mean_fpt"], out["kramers_tau"])
    assert sum(out["censored"]) == 0
    assert out["delta_U_arrhenius"] == pytest.approx(du, rel=0.08)
    for tau, kt in zip(out["mean_fpt"], out["kramers_tau"]):
        assert tau == pytest.approx(kt, rel=0.25)


def _fd_mean(alpha, T, ramp, **kw):
    g = np.linspace(0.0, 0.999, 20000)
    P = analysis.fulton_dunkleberger_cdf(g, alpha, T, ramp, **kw)
    return float(np.sum(1.0 - P) * (g[1] - g[0]))  # E[gamma_sw] = int (1 - P)


@pytest.mark.parametrize("scheme", [1, 0])
def test_switching_cdf_matches_adiabatic_theory(scheme):
    # Li07 damping and temperature.  The semi-implicit scheme (1) samples the
    # well at T (to 1e-4 at dt = 0.02) and is held to the theory.  The
    # explicit scheme (0) heats the well bottom to 1.064 T, less at the higher
    # energies escape passes through: its mean switching bias lies between
    # the theory at 1.064 T and the theory at T.
    a, T, ramp, dt = 0.283, 0.0673, 1e-6, 0.02
    out = analysis.switching_distribution(alpha=a, T=T, ramp=ramp, n_replicas=30000,
                                          dt=dt, scheme=scheme)
    m = out["mean_gamma_sw"]
    m_t = _fd_mean(a, T, ramp)
    m_hot = _fd_mean(a, T, ramp, dt=dt, scheme=0)
    print(f"scheme {scheme}: max |CDF - FD(T)| = {out['max_abs_diff']:.4f}, mean gamma_sw "
          f"{m:.5f}, FD mean at T {m_t:.5f}, at the heated well {m_hot:.5f}")
    assert out["gamma_sw"].size == 30000
    se = float(np.std(out["gamma_sw"])) / np.sqrt(30000)
    if scheme == 1:
        assert out["max_abs_diff"] < 0.05
    else:
        assert m_hot + 3 * se < m < m_t - 3 * se
