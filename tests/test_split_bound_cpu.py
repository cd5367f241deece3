"""CPU check of the error model behind the split half-precision product
(ns_gemm_f32_split) and the tolerance its GPU tests use.

A float32 matrix X is scaled by 2^e, e = 14 - floor(log2 max|X|) (so the
largest magnitude lands in [2^14, 2^15)), and split into IEEE half-precision
planes hi = half(x 2^e), lo = half(x 2^e - hi).  The model here is numpy's
float16 rounding (round to nearest even, subnormals kept), written from that
definition; it shares no code with the library.  Checked:

* representation: |x - (hi + lo) 2^-e| <= 2^-22 |x| + 2^-25 2^-e for every
  element (half-precision subnormal step 2^-24 below 2^-14), over magnitudes
  spread across 2^-60 .. 2^20;
* x 2^e - hi is exact in float32 (the split loses nothing before lo is
  rounded);
* the three-product sum hi hi' + hi lo' + lo hi', accumulated exactly (float64
  here), stays within 3 2^-22 |X||Y| + 2^-38 (max|X| sum|Y| + max|Y| sum|X|)
  of X Y -- the accumulation-free part of the bound in test_gpu_lowp.split_bound.
"""
import numpy as np
import pytest


def split(x32):
    m = float(np.max(np.abs(x32)))
    e = 0 if not (0.0 < m < np.inf) else 14 - int(np.floor(np.log2(m)))
    e = max(-100, min(100, e))
    xs = (x32.astype(np.float64) * 2.0 ** e).astype(np.float32)   # exact: power of two
    hi = xs.astype(np.float16)
    with np.errstate(invalid="ignore"):          # inf - inf for non-finite input
        rem32 = xs - hi.astype(np.float32)
    lo = rem32.astype(np.float16)
    return e, xs, hi, lo, rem32


def spread(rng, shape, lo=-60, hi=20):
    x = rng.standard_normal(shape).astype(np.float32)
    return (x * np.exp2(rng.integers(lo, hi + 1, shape)).astype(np.float32)).astype(np.float32)


@pytest.mark.parametrize("seed", range(6))
def test_split_representation_bound(seed):
    rng = np.random.default_rng(seed)
    x = spread(rng, (300, 200)) if seed % 2 else rng.standard_normal((300, 200)).astype(np.float32)
    e, xs, hi, lo, rem32 = split(x)
    scaled_max = float(np.max(np.abs(xs)))
    assert 2.0 ** 14 <= scaled_max < 2.0 ** 15
    # the remainder is exact in float32
    assert np.array_equal(rem32.astype(np.float64),
                          xs.astype(np.float64) - hi.astype(np.float64))
    rec = (hi.astype(np.float64) + lo.astype(np.float64)) * 2.0 ** -e
    err = np.abs(x.astype(np.float64) - rec)
    bound = 2.0 ** -22 * np.abs(x.astype(np.float64)) + 2.0 ** -25 * 2.0 ** -e
    assert np.all(err <= bound), float(np.max(err / bound))
    # hi never overflows half precision
    assert np.all(np.isfinite(hi)) and np.all(np.isfinite(lo))


@pytest.mark.parametrize("seed", range(4))
def test_three_product_bound(seed):
    rng = np.random.default_rng(100 + seed)
    m, k, n = 40, 300, 30
    X = spread(rng, (m, k), -40, 10)
    Y = rng.standard_normal((k, n)).astype(np.float32) * np.float32(1e-3)
    ex, _, xh, xl, _ = split(X)
    ey, _, yh, yl, _ = split(Y)
    xh, xl = xh.astype(np.float64), xl.astype(np.float64)
    yh, yl = yh.astype(np.float64), yl.astype(np.float64)
    approx = (xh @ yh + xh @ yl + xl @ yh) * 2.0 ** -(ex + ey)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    ref = Xd @ Yd
    ax, ay = np.abs(Xd), np.abs(Yd)
    bound = (3 * 2.0 ** -22 * (ax @ ay)
             + 2.0 ** -38 * (ax.max() * ay.sum(axis=0)[None, :] + ay.max() * ax.sum(axis=1)[:, None]))
    assert np.all(np.abs(approx - ref) <= bound), float(np.max(np.abs(approx - ref) / bound))


def test_degenerate_scales():
    # a zero matrix keeps exponent 0; a non-finite maximum does too
    e, *_ = split(np.zeros((4, 4), np.float32))
    assert e == 0
    x = np.ones((4, 4), np.float32)
    x[1, 2] = np.inf
    e, *_ = split(x)
    assert e == 0
    # the exponent is clamped for vanishing matrices
    e, *_ = split(np.full((2, 2), 1e-38, np.float32))
    assert e == 100
