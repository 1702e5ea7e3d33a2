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
