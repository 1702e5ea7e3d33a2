"""Host-side theory of the analysis module (no GPU): barrier height against
the value the paper prints, the Kramers rate against the pinned oracle
formula, and the Fulton-Dunkleberger CDF's limits."""

import json
import math
import os

import numpy as np
import pytest

from paper_1802_05065_amd import analysis

HERE = os.path.dirname(os.path.abspath(__file__))


def test_barrier_height_paper_value():
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["arrhenius_fig"]
    du = analysis.barrier_height(g["gamma"], V0=g["amplitude_as_printed"])
    assert float(du) == pytest.approx(g["delta_U_theory"], abs=5e-5)
    assert float(analysis.barrier_height(0.0)) == pytest.approx(2.0)
    assert float(analysis.barrier_height(1.0)) == pytest.approx(0.0, abs=1e-12)


def test_kramers_rate_closed_form():
    g, a, T = 0.8, 0.5, 0.034
    w = (1 - g * g) ** 0.25
    lam = math.sqrt(a * a / 4 + w * w) - a / 2
    du = 2 * (math.sqrt(1 - g * g) - g * math.acos(g))
    ref = w / (2 * math.pi) * lam / w * math.exp(-du / T)
    assert float(analysis.kramers_rate(g, a, T)) == pytest.approx(ref, rel=1e-12)
    # V0 scales the frequencies by sqrt(V0) and the barrier by V0
    r2 = float(analysis.kramers_rate(g, a, T * 4.0, V0=4.0))
    w2 = 2 * w
    lam2 = math.sqrt(a * a / 4 + w2 * w2) - a / 2
    assert r2 == pytest.approx(w2 / (2 * math.pi) * lam2 / w2 * math.exp(-du / T), rel=1e-12)


def test_fulton_dunkleberger_cdf_limits():
    g = np.linspace(0, 0.999, 2000)
    P = analysis.fulton_dunkleberger_cdf(g, 0.283, 0.0673, 1e-6)
    assert P[0] == 0.0
    assert np.all(np.diff(P) >= 0)
    assert P[-1] == pytest.approx(1.0, abs=1e-9)
    # slower ramps switch earlier
    slow = analysis.fulton_dunkleberger_cdf(g, 0.283, 0.0673, 1e-8)
    assert np.all(slow >= P - 1e-12)


@pytest.mark.parametrize("power", [0, -1])
def test_barrier_fits_recover_the_exponent(power):
    # tau = A T^power exp(dU / T): the Arrhenius slope (ln tau vs 1/T) is dU
    # for power 0, the prefactor form (ln(T tau) vs 1/T) is dU for power -1
    du, A = 0.0342, 37.0
    T = du / np.array([3.5, 4.5, 5.5, 6.5])
    tau = A * T ** power * np.exp(du / T)
    se = 0.014 * tau
    fits = analysis.barrier_fits(T, tau, se)
    exact = "delta_U_arrhenius" if power == 0 else "delta_U_kramers_form"
    assert fits[exact] == pytest.approx(du, rel=1e-12)
    # the other form differs by the slope of ln T against 1/T
    other = "delta_U_kramers_form" if power == 0 else "delta_U_arrhenius"
    ln_t_slope = np.polyfit(1.0 / T, np.log(T), 1)[0]
    assert fits[other] - fits[exact] == pytest.approx(ln_t_slope if power == 0 else -ln_t_slope,
                                                      rel=1e-9)
    # standard error of a weighted slope against numpy's covariance
    rng = np.random.Generator(np.random.PCG64(3))
    noisy = tau * np.exp(rng.normal(0, 0.014, size=4))
    f2 = analysis.barrier_fits(T, noisy, 0.014 * noisy)
    coef, cov = np.polyfit(1.0 / T, np.log(noisy), 1, w=1.0 / np.full(4, 0.014), cov="unscaled")
    assert f2["delta_U_arrhenius"] == pytest.approx(coef[0], rel=1e-9)
    assert f2["delta_U_arrhenius_se"] == pytest.approx(math.sqrt(cov[0, 0]), rel=1e-9)
