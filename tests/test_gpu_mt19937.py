"""GPU parity of the MT19937 mode (Algorithm 2's generator): the words, the
trajectories and the escape steps of the HIP path against the oracle, and the
results' independence of the launch shape (the generator state is resident in
device memory between launches)."""

import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1802_05065_amd import api, workloads

pytestmark = pytest.mark.gpu

FIXED = dict(replicas_per_lane=1, waves_per_simd=4, steps_per_launch=4096)
INT_MOMENTS = ("n_escaped", "n_censored", "n_overflow", "sum_k", "sum_k2")


def _op(p):
    return oracle.OracleParams(**workloads.to_oracle_kwargs(p))


def _steps(res, i=0):
    return res.steps[i].cpu().numpy()


def test_mt_words_bit_exact():
    # 170 blocks = 680 words: crosses the first 624-word regeneration
    w = api.mt_words(seed=5489, replica0=0, n_rep=8, block0=0, n_blk=170)
    for r in range(8):
        ref = oracle.mt19937(5489 + r, 170 * 4).reshape(170, 4)
        assert np.array_equal(w[r], ref), r
    # seed + replica wraps modulo 2^32; a window past the second regeneration
    w2 = api.mt_words(seed=2**32 - 2, replica0=0, n_rep=4, block0=300, n_blk=20)
    for r in range(4):
        ref = oracle.mt19937((2**32 - 2 + r) % 2**32, 320 * 4).reshape(320, 4)[300:]
        assert np.array_equal(w2[r], ref), r
    # ragged replica count (not a multiple of the 64-lane launch)
    w3 = api.mt_words(seed=11, replica0=1000, n_rep=67, block0=0, n_blk=2)
    assert np.array_equal(w3[66], oracle.mt19937(11 + 1066, 8).reshape(2, 4))


@pytest.mark.parametrize("model", ["underdamped", "overdamped"])
def test_mt_trajectory_fp64_matches_oracle(model):
    maker = workloads.plain_escape if model == "underdamped" else workloads.uneven_overdamped
    p = dict(maker(n_replicas=4), threshold=1e300, rng=1)
    phi, v = api.trajectory(p, replica=3, n_steps=3001, precision="fp64")
    rphi, rv = oracle.trajectory(_op(p), 3, 3001)
    np.testing.assert_allclose(phi, rphi, rtol=0, atol=1e-9)
    np.testing.assert_allclose(phi[:50], rphi[:50], rtol=1e-15, atol=0)
    if p["model"] == 0:
        np.testing.assert_allclose(v, rv, rtol=0, atol=1e-9)


def test_mt_escape_steps_match_oracle():
    p = dict(workloads.plain_escape(n_replicas=3000, seed=77), rng=1)
    ref = oracle.escape_steps(_op(p), 0, p["n_replicas"])
    for t in (FIXED, dict(schedule=1, replicas_per_lane=1, steps_per_launch=2048)):
        res = api.simulate(p, "fp64", t)
        gpu = _steps(res)
        same = np.mean(gpu == ref)
        print(f"MT19937 identical FP64 escape steps ({t}): {same:.5f}")
        assert same >= 0.99
        h, m = oracle.histogram(gpu, p["n_bins"], p["hist_k_max"], p["dt"])
        assert res.counts[0].tolist() == h.tolist()
        for k in INT_MOMENTS:
            assert res.moments[0][k] == m[k], k


def test_mt_results_independent_of_launch_shape():
    # short launches: every lane restores its generator mid-regeneration
    p = dict(workloads.uneven_overdamped(n_replicas=5000, seed=8), max_steps=40_001, rng=1)
    tunings = [dict(replicas_per_lane=1, waves_per_simd=8, steps_per_launch=1024),
               dict(replicas_per_lane=1, waves_per_simd=1, steps_per_launch=68),
               dict(schedule=1, replicas_per_lane=1, steps_per_launch=2000),
               dict(replicas_per_lane=1, waves_per_simd=2, steps_per_launch=512, use_graph=1)]
    for prec in ("fp64", "fp32c"):
        base = api.simulate(p, prec, tunings[0])
        b = _steps(base)
        assert (b == -1).any() and (b > 0).any()
        for t in tunings[1:]:
            r = api.simulate(p, prec, t)
            assert np.array_equal(_steps(r), b), (prec, t)
            assert r.counts[0].tolist() == base.counts[0].tolist()
    idx = np.arange(0, 5000, 250)
    b64 = _steps(api.simulate(p, "fp64", tunings[0]))
    ref = np.array([oracle.escape_steps(_op(p), int(i), 1)[0] for i in idx])
    assert np.mean(b64[idx] == ref) >= 0.99


def test_mt_and_philox_give_the_same_distribution():
    n = 2 ** 14
    p = workloads.plain_escape(n_replicas=n, seed=300)
    s_mt = _steps(api.simulate(dict(p, rng=1), "fp32c", FIXED))
    s_ph = _steps(api.simulate(dict(p, seed=301), "fp32c", FIXED))
    assert (s_mt > 0).all() and (s_ph > 0).all()
    ks = stats.ks_2samp(s_mt, s_ph)
    se = math.sqrt(s_mt.var() / n + s_ph.var() / n)
    print(f"MT vs Philox: KS p = {ks.pvalue:.3f}, means {s_mt.mean():.1f} {s_ph.mean():.1f}")
    assert ks.pvalue > 0.01
    assert abs(s_mt.mean() - s_ph.mean()) < 3 * se
