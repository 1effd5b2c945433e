"""Pins of the oracle's windowed quantiles (Section 3.4's sliding histograms).

The paper does not define which quantile it means; the oracle uses the inverse
empirical CDF (rho-th smallest value, rho = max(1, ceil(q n))).  That choice is
"parity unpinned" as a reading of the paper, but the computation itself is
pinned here against sorting, SciPy's order-statistic filters and closed forms.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import brute
from docgen import gen_document


def _rand(H, W, seed, hi=256):
    return np.random.default_rng(seed).integers(0, hi, size=(H, W), dtype=np.uint8)


def test_rank_rule():
    assert oracle.rank(0.5, 9) == 5
    assert oracle.rank(0.5, 10) == 5          # lower median for even n
    assert oracle.rank(0.1, 1024) == 103      # ceil(102.4)
    assert oracle.rank(0.0, 7) == 1           # the minimum
    assert oracle.rank(1.0, 7) == 7           # the maximum
    assert oracle.rank(1e-9, 5) == 1


def test_pure_python_tiny():
    rng = np.random.default_rng(2)
    for (H, W, h, w, q) in [(6, 7, 3, 4, 0.5), (5, 5, 2, 2, 0.1), (4, 9, 6, 3, 0.9), (1, 5, 4, 4, 0.5)]:
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        ref = brute.quantile_python(I, h, w, q)
        a, _ = oracle.quantile_sort(I, h, w, q)
        b, _ = oracle.quantile_hist(I, h, w, q)
        assert np.array_equal(a, ref) and np.array_equal(b, ref)


def test_sort_equals_histogram_many():
    for seed, (H, W, h, w, q) in enumerate([(40, 50, 9, 9, 0.5), (37, 61, 8, 12, 0.1),
                                            (64, 64, 32, 32, 0.5), (50, 30, 101, 101, 0.1),
                                            (25, 70, 1, 1, 0.5), (45, 45, 16, 5, 0.75)]):
        I = gen_document(H, W, seed + 10, noise=10, stain=True)
        a, ma = oracle.quantile_sort(I, h, w, q)
        b, mb = oracle.quantile_hist(I, h, w, q)
        assert np.array_equal(a, b) and np.array_equal(ma, mb)
        assert np.array_equal(ma, (I < a).astype(np.uint8))


def _scipy_origin(h, w, fn):
    """Origin that makes SciPy's filter window equal the oracle's, found from
    the impulse response (for even sizes the two conventions differ by one)."""
    H, W = 3 * h + 3, 3 * w + 3
    a, b = H // 2, W // 2
    I = np.zeros((H, W), np.uint8)
    I[a, b] = 1
    o, u, l, r = oracle.extents(h, w)
    want = np.zeros((H, W), np.uint8)
    want[a - u:a + o, b - r:b + l] = 1
    for oy in (0, -1, 1):
        for ox in (0, -1, 1):
            got = fn(I, size=(h, w), mode="nearest", origin=(oy, ox))
            if np.array_equal(got, want):
                return (oy, ox)
    raise AssertionError("no SciPy origin reproduces the window")


@pytest.mark.parametrize("h,w", [(5, 7), (4, 6), (8, 3), (1, 2)])
def test_min_max_equal_scipy_filters(h, w):
    # With clipping, the window min/max equal the 'nearest'-padded filters
    # (replicated border values already lie in the window).
    I = _rand(41, 53, h * 10 + w)
    org = _scipy_origin(h, w, ndimage.maximum_filter)
    qmax, _ = oracle.quantile_hist(I, h, w, 1.0)
    qmin, _ = oracle.quantile_hist(I, h, w, 0.0)
    assert np.array_equal(qmax, ndimage.maximum_filter(I, size=(h, w), mode="nearest", origin=org))
    assert np.array_equal(qmin, ndimage.minimum_filter(I, size=(h, w), mode="nearest", origin=org))


@pytest.mark.parametrize("h,w,q", [(7, 7, 0.5), (9, 5, 0.1), (6, 8, 0.5), (11, 11, 0.9)])
def test_interior_rank_filter(h, w, q):
    # Interior pixels (full windows, n = h w) equal SciPy's rank filter.
    I = gen_document(60, 70, 5, noise=10, stain=True)
    org = _scipy_origin(h, w, ndimage.maximum_filter)
    n = h * w
    rho = oracle.rank(q, n)
    ref = ndimage.rank_filter(I, rank=rho - 1, size=(h, w), mode="nearest", origin=org)
    got, _ = oracle.quantile_hist(I, h, w, q)
    o, u, l, r = oracle.extents(h, w)
    inner = (slice(o - 1, 60 - u), slice(l - 1, 70 - r))
    assert np.array_equal(got[inner], ref[inner])
    if q == 0.5 and n % 2 == 1:
        med = ndimage.median_filter(I, size=(h, w), mode="nearest", origin=org)
        assert np.array_equal(got[inner], med[inner])


def test_constant_and_monotone():
    I = np.full((20, 20), 77, np.uint8)
    Q, mask = oracle.quantile_hist(I, 5, 5, 0.3)
    assert np.all(Q == 77) and not mask.any()
    J = gen_document(50, 50, 3, noise=10)
    prev = None
    for q in (0.0, 0.1, 0.25, 0.5, 0.75, 0.9, 1.0):
        Q, _ = oracle.quantile_hist(J, 8, 8, q)
        if prev is not None:
            assert np.all(Q >= prev)
        prev = Q
