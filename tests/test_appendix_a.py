"""Pins of the Appendix A parallel-execution model (oracle/appendix_a.py):
closed forms for one run per thread (maximum of N unit exponentials has mean
H_N) and one thread (Erlang mean N_L), and a Monte Carlo check otherwise."""

import math

import numpy as np
import pytest

from oracle import appendix_a


@pytest.mark.parametrize("n", [1, 2, 20, 64, 512])
def test_one_run_per_thread_is_harmonic_number(n):
    h = sum(1.0 / i for i in range(1, n + 1))
    assert appendix_a.mean_parallel_time(n, 1) == pytest.approx(h, rel=1e-7)
    assert appendix_a.efficiency(n, 1) == pytest.approx(1.0 / h, rel=1e-7)


@pytest.mark.parametrize("nl", [1, 3, 50])
def test_single_thread_is_perfect(nl):
    assert appendix_a.efficiency(1, nl) == pytest.approx(1.0, rel=1e-7)


@pytest.mark.parametrize("n,nl", [(64, 4), (20, 16), (64, 64)])
def test_monte_carlo(n, nl):
    rng = np.random.Generator(np.random.PCG64(1))
    m = rng.gamma(nl, 1.0, size=(20000, n)).max(axis=1)
    ref = m.mean()
    se = m.std() / math.sqrt(m.size)
    assert appendix_a.mean_parallel_time(n, nl) == pytest.approx(ref, abs=4 * se)


def test_efficiency_grows_with_load():
    e = [appendix_a.efficiency(64, nl) for nl in (1, 2, 8, 64, 256)]
    assert all(a < b for a, b in zip(e, e[1:]))
    assert e[0] == pytest.approx(0.211, abs=0.001)
