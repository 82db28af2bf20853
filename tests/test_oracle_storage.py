"""Pins for the oracle's FP32 base distance (fixed lane order) and for the
bfloat16 / binary16 storage conversions of the precision form.

Library pins: numpy's float16 and torch's bfloat16 conversions (both round
to nearest even). Exactness pins: on integer data every summation order is
exact, so the base keys equal the FP64 sums. Order pins: hand-computed
cases where the lane order decides the rounding.
"""
import numpy as np
import pytest
import torch

import oracle


def _edge_floats():
    rng = np.random.Generator(np.random.PCG64(9))
    vals = [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.99, 65520.0, 65536.0, 1e-8, 6.1e-5, 5.96e-8,
            2.98e-8, 2.99e-8, 3.4e38, -3.4e38, 1.0 + 2 ** -11, 1.0 + 2 ** -10 + 2 ** -11,
            np.inf, -np.inf]
    r = np.concatenate([np.array(vals, np.float64),
                        rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000)])
    # exact halfway cases for binary16 and bfloat16
    mids16 = (np.arange(1, 2000, dtype=np.float64) + 0.5) * 2.0 ** -10
    midsbf = (np.arange(1, 2000, dtype=np.float64) + 0.5) * 2.0 ** -7
    return np.concatenate([r, mids16, -mids16, midsbf]).astype(np.float32)


def test_f16_matches_numpy():
    x = _edge_floats()
    got = oracle.convert(x, oracle.F16)
    ref = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_bf16_matches_torch():
    x = _edge_floats()
    got = oracle.convert(x, oracle.BF16)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_widen_exact():
    x = _edge_floats()[:3000]
    h16 = oracle.convert(x, oracle.F16)
    np.testing.assert_array_equal(oracle.widen(h16, oracle.F16), h16.view(np.float16).astype(np.float32))
    hb = oracle.convert(x, oracle.BF16)
    ref = torch.from_numpy(hb.view(np.int16)).view(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(oracle.widen(hb, oracle.BF16), ref)


@pytest.mark.parametrize("g,v", [(1, 1), (8, 4), (16, 4), (32, 4), (64, 4), (16, 2), (64, 1)])
def test_base_dist_integer_exact(g, v):
    rng = np.random.Generator(np.random.PCG64(10))
    for d in (1, 7, 32, 100, 128, 960):
        x = rng.integers(0, 256, size=d).astype(np.float32)
        q = rng.integers(0, 256, size=d).astype(np.float32)
        dl = (x.astype(np.int64) - q.astype(np.int64))
        assert oracle.base_dist(x, q, 1, g, v) == float(np.abs(dl).sum())
        assert oracle.base_dist(x, q, 2, g, v) == float((dl * dl).sum())


@pytest.mark.parametrize("g,v", [(1, 1), (8, 4), (16, 4), (64, 4), (16, 2)])
def test_base_dist_l05_perfect_squares_exact(g, v):
    """L0.5 base key sum sqrt|x - q|: with |x - q| a perfect square every
    root is an exact integer and every partial sum too, so the key is the
    integer sum in any order."""
    rng = np.random.Generator(np.random.PCG64(12))
    for d in (1, 7, 32, 128, 960):
        r = rng.integers(0, 16, size=d)
        q = rng.integers(0, 256, size=d).astype(np.float64)
        sign = np.where(rng.random(d) < 0.5, -1.0, 1.0)
        x = (q + sign * r * r).astype(np.float32)
        assert oracle.base_dist(x, q.astype(np.float32), oracle.L05, g, v) == float(r.sum())


def test_base_dist_l05_error_bound_and_rank():
    """Against sum sqrt|x - q| in FP64: each correctly rounded root adds at
    most u relative, the sum gamma_k as above. Rank pin: the key's square is
    the L0.5 distance of the FP64 definition (oracle.lp_dist at p = 0.5)."""
    rng = np.random.Generator(np.random.PCG64(13))
    u = 2.0 ** -24
    for d, g in ((32, 8), (128, 32), (960, 64), (100, 16)):
        x = rng.standard_normal(d).astype(np.float32)
        q = rng.standard_normal(d).astype(np.float32)
        exact = np.sqrt(np.abs(x.astype(np.float64) - q.astype(np.float64))).sum()
        kk = -(-d // g) + 4 + int(np.log2(g)) + 3
        got = oracle.base_dist(x, q, oracle.L05, g, 4)
        assert abs(got - exact) <= kk * u * exact * 1.01
        assert abs(got * got - oracle.lp_dist(x, q, 0.5)) <= 2.1 * kk * u * exact * exact


def test_base_dist_l05_rounded_root():
    """The root is taken in FP32, correctly rounded, per element: |x - q| = 2
    gives fl(sqrt 2) = 1.41421353816986083984375 (not the FP64 root 1.41421356...)."""
    x = np.array([2.0], np.float32)
    q = np.zeros(1, np.float32)
    assert oracle.base_dist(x, q, oracle.L05, 1, 1) == float(np.sqrt(np.float32(2.0)))
    assert oracle.base_dist(x, q, oracle.L05, 1, 1) == 1.41421353816986083984375
    # two lanes (g = 2, v = 1): lane sums sqrt2 and sqrt3, then one rounded add
    x2 = np.array([2.0, 3.0], np.float32)
    want = float(np.float32(np.sqrt(np.float32(2.0))) + np.float32(np.sqrt(np.float32(3.0))))
    assert oracle.base_dist(x2, np.zeros(2, np.float32), oracle.L05, 2, 1) == want


def test_base_dist_error_bound():
    """|fl(delta) - delta| <= gamma_k * sum|terms|, k = ceil(d/g) + v + log2 g + 2."""
    rng = np.random.Generator(np.random.PCG64(11))
    u = 2.0 ** -24
    for d, g in ((32, 8), (128, 32), (960, 64), (100, 16)):
        x = rng.standard_normal(d).astype(np.float32)
        q = rng.standard_normal(d).astype(np.float32)
        dl = x.astype(np.float64) - q.astype(np.float64)
        kk = -(-d // g) + 4 + int(np.log2(g)) + 2
        for metric, exact in ((1, np.abs(dl).sum()), (2, (dl * dl).sum())):
            got = oracle.base_dist(x, q, metric, g, 4)
            assert abs(got - exact) <= kk * u * exact * 1.01


def test_base_dist_lane_order():
    """Hand-computed: terms [2^24, 1, 1, 1].
    Sequential (g=1): ((2^24+1)+1)+1 rounds to 2^24 at every step.
    g=2, v=1: lane0 = 2^24+1 -> 2^24, lane1 = 1+1 = 2, total 2^24+2.
    g=2, v=2: lane0 = 2^24+1 -> 2^24 (elements 0,1), lane1 = 2 (elements 2,3)."""
    x = np.array([2.0 ** 24, 1, 1, 1], np.float32)
    q = np.zeros(4, np.float32)
    assert oracle.base_dist(x, q, 1, 1, 1) == 16777216.0
    assert oracle.base_dist(x, q, 1, 2, 1) == 16777218.0
    assert oracle.base_dist(x, q, 1, 2, 2) == 16777218.0
    # g=4, v=1: lanes hold 2^24, 1, 1, 1; o=2: (2^24+1)->2^24, (1+1)=2; o=1: 2^24+2
    assert oracle.base_dist(x, q, 1, 4, 1) == 16777218.0
    # terms [1, 2^24, 1, 1] with g=2, v=1: lane0 = 1+1 = 2, lane1 = 2^24+1 -> 2^24; sum 2^24+2
    x2 = np.array([1, 2.0 ** 24, 1, 1], np.float32)
    assert oracle.base_dist(x2, q, 1, 2, 1) == 16777218.0
    # sequential on x2: 1 + 2^24 = 2^24+1 -> 2^24 (ties to even), +1 -> 2^24, +1 -> 2^24
    assert oracle.base_dist(x2, q, 1, 1, 1) == 16777216.0
    # v = 4, g = 2: elements 0..3 go to lane 0, 4..7 to lane 1. Terms [2^24,1,1,1,0,0,0,0]:
    # lane 0 absorbs every +1 (2^24 each step), lane 1 = 0, total 2^24. (Had elements
    # been dealt round-robin, lane 1 would hold 1+1 = 2 and the total 2^24+2.)
    x3 = np.array([2.0 ** 24, 1, 1, 1, 0, 0, 0, 0], np.float32)
    q8 = np.zeros(8, np.float32)
    assert oracle.base_dist(x3, q8, 1, 2, 4) == 16777216.0
    assert oracle.base_dist(x3, q8, 1, 2, 1) == 16777218.0


def test_base_dist_fma():
    """L2 accumulates with a fused multiply-add, which rounds once.
    Terms (g = 1): x = [2^-12, 2^-12, 1 + 2^-12], q = 0.
    s = fma(2^-12, 2^-12, 0) = 2^-24; s = fma(2^-12, 2^-12, s) = 2^-23;
    (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 exactly, so the fused step rounds
    1 + 2^-11 + 3*2^-24 (1.5 ulp past 1 + 2^-11, a tie) to even: 1 + 2^-11 + 2^-22.
    Unfused, the square rounds first to 1 + 2^-11 (tie to even) and the sum is
    1 + 2^-11 + 2^-23."""
    x = np.array([2.0 ** -12, 2.0 ** -12, 1 + 2.0 ** -12], np.float32)
    q = np.zeros(3, np.float32)
    fused = np.float32(1 + 2 ** -11 + 2 ** -22)
    unfused = np.float32(1 + 2 ** -11 + 2 ** -23)
    assert fused != unfused
    assert oracle.base_dist(x, q, 2, 1, 1) == fused
