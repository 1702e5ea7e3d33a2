"""The FP32C phase arithmetic, emulated in IEEE float32 on the host.

Between 4-step blocks the phase is a float pair (phr, e); inside a block a
float running sum d starts at e and takes the 4 increments, and the block's
end forms t = phr + d rounded and e' = d - (t - phr).  These tests check the
two facts the scheme rests on: the fold loses nothing (t + e' equals
phr + d exactly when |phr| >= |d|, the Fast2Sum condition), and over many
blocks the pair tracks the exact sum of the increments far more closely than
plain float32 accumulation does."""

import numpy as np

f32 = np.float32


def fold(phr, d):
    t = f32(phr + d)
    return t, f32(d - f32(t - phr))


def test_fold_is_exact_under_fast2sum_condition():
    rng = np.random.default_rng(7)
    phr = rng.uniform(-1.5, 1.5, 200_000).astype(np.float32)
    d = (rng.uniform(-1.0, 1.0, phr.size) * np.abs(phr)).astype(np.float32)
    t = (phr + d).astype(np.float32)
    e = (d - (t - phr).astype(np.float32)).astype(np.float32)
    exact = phr.astype(np.float64) + d.astype(np.float64)
    assert np.array_equal(t.astype(np.float64) + e.astype(np.float64), exact)


def test_block_compensated_sum_tracks_exact_sum():
    # a phase drifting over 1.2 revolutions in increments of ~1e-4 revolution
    # (the size of a switching replica's steps near the barrier)
    rng = np.random.default_rng(11)
    n_blocks = 100_000
    inc = (rng.normal(3e-6, 1e-4, (n_blocks, 4))).astype(np.float32)
    phr, e = f32(0.0), f32(0.0)
    plain = f32(0.0)
    exact = 0.0
    worst_pair = worst_plain = 0.0
    for blk in range(n_blocks):
        d = e
        for q in range(4):
            d = f32(d + inc[blk, q])
            plain = f32(plain + inc[blk, q])
            exact += float(inc[blk, q])
        phr, e = fold(phr, d)
        worst_pair = max(worst_pair, abs(float(phr) + float(e) - exact))
        worst_plain = max(worst_plain, abs(float(plain) - exact))
    # the pair's error stays at the level of the running sums' own rounding
    # (a few 2^-24 of an increment per block, random in sign), far below
    # plain accumulation's
    assert worst_pair < 1e-8, worst_pair
    assert worst_plain > 50 * worst_pair, (worst_plain, worst_pair)
