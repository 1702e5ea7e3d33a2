"""Appendix A of arXiv:1802.05065: the statistical model of parallel execution.

TEST INFRASTRUCTURE ONLY (used to assess the measured lane utilisation of the
one-replica-per-lane and refill schedules).

Model (Appendix A, Eqs. (A.1)-(A.5)): each run's execution time is an
exponential deviate with unit mean; a thread that executes N_L runs one after
the other takes an Erlang(N_L, 1) time; with N_tpb threads working in parallel
the parallel time is the maximum of N_tpb independent Erlang(N_L, 1) times, so
its CDF is the Erlang CDF raised to the power N_tpb.  The speed-up is
S = <E_t>/<E_p> with <E_t> = N_r = N_L N_tpb, and the efficiency is S/N_tpb.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def mean_parallel_time(n_threads: int, n_load: int) -> float:
    """<E_p> = integral_0^inf (1 - CDF_Erlang(N_L,1)(x)^N_tpb) dx."""
    if n_threads < 1 or n_load < 1:
        raise ValueError("n_threads and n_load must be >= 1")

    def tail(x: float) -> float:
        return 1.0 - special.gammainc(n_load, x) ** n_threads

    # the integrand is ~1 up to the bulk of the maximum, then decays like
    # N_tpb * Erlang tail; integrate piecewise up to where it is negligible
    upper = n_load + 20.0 * math.sqrt(n_load) + 3.0 * math.log(n_threads) + 60.0
    knots = np.linspace(0.0, upper, 65)
    total = 0.0
    for a, b in zip(knots[:-1], knots[1:]):
        total += integrate.quad(tail, a, b, limit=200)[0]
    return total


def speedup(n_threads: int, n_load: int) -> float:
    """S = <E_t>/<E_p> with <E_t> = N_L * N_tpb (Eq. (A.5))."""
    return n_load * n_threads / mean_parallel_time(n_threads, n_load)


def efficiency(n_threads: int, n_load: int) -> float:
    """S / N_tpb: 1 for a perfectly balanced parallel run."""
    return speedup(n_threads, n_load) / n_threads
