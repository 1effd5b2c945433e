"""Pins of the oracle's window geometry, counts and window sums.

Each check ties the C oracle to something other than itself: the window read
straight off the Introduction's inequality (pure Python / shifted images), the
paper's three implementations agreeing (direct, integral images, recursive
Algorithm 1; Section 4), closed forms and invariants.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from docgen import gen_document


def _rand(H, W, seed, hi=256):
    return np.random.default_rng(seed).integers(0, hi, size=(H, W), dtype=np.uint8)


def test_extents_match_introduction_bounds():
    # Algorithm 1's o, u, l, r describe the Introduction's window
    # i - h/2 < a <= i + h/2 for every size, odd and even.
    for size in range(1, 260):
        o, u, l, r = oracle.extents(size, size)
        offs = brute.window_offsets(size)
        assert offs == list(range(-o + 1, u + 1))
        assert offs == list(range(-l + 1, r + 1))
        assert len(offs) == size


def test_pure_python_brute_force_tiny():
    rng = np.random.default_rng(7)
    for (H, W, h, w) in [(5, 7, 4, 3), (6, 4, 2, 5), (3, 3, 9, 8), (1, 6, 3, 2), (7, 1, 6, 1)]:
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        S1p, S2p, Np = brute.sums_python(I, h, w)
        S1, S2 = oracle.sums_direct(I, h, w)
        assert np.array_equal(S1.astype(np.int64), S1p)
        assert np.array_equal(S2.astype(np.int64), S2p)
        assert np.array_equal(oracle.count_map(H, W, h, w), Np)


def test_exhaustive_tiny_sweep_three_implementations():
    # H, W in 1..12 and h, w in 1..9 (windows larger than the image included):
    # direct, recursive and integral-image sums all equal the shifted-image sum.
    rng = np.random.default_rng(11)
    for H in range(1, 13):
        for W in range(1, 13):
            I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
            for h in range(1, 10):
                for w in range(1, 10):
                    ref1, ref2 = brute.sums_shift(I, h, w)
                    for fn in (oracle.sums_direct, oracle.sums_recursive, oracle.sums_integral):
                        a, b = fn(I, h, w)
                        assert np.array_equal(a.astype(np.int64), ref1), (fn.__name__, H, W, h, w)
                        assert np.array_equal(b.astype(np.int64), ref2), (fn.__name__, H, W, h, w)


def test_count_formula_equals_counting():
    for (H, W, h, w) in [(1, 1, 1, 1), (9, 13, 4, 7), (20, 3, 32, 2), (31, 17, 8, 8)]:
        n = oracle.count_map(H, W, h, w)
        assert np.array_equal(n, brute.count_shift(H, W, h, w))
        # the all-ones image has S1 = n (Algorithm 1's n)
        S1, S2 = oracle.sums_recursive(np.ones((H, W), np.uint8), h, w)
        assert np.array_equal(S1.astype(np.int64), n)
        assert np.array_equal(S2.astype(np.int64), n)
        for (i, j) in [(0, 0), (H - 1, W - 1), (H // 2, W // 3)]:
            assert oracle.count(H, W, h, w, i, j) == n[i, j]


@pytest.mark.parametrize("h,w", [(1, 1), (2, 2), (3, 4), (4, 3), (6, 5), (32, 32), (15, 8)])
def test_impulse_response_is_reflected_window(h, w):
    # A single 1 at (a, b) contributes to exactly the pixels whose window holds
    # (a, b): rows a-u .. a+o-1 and columns b-r .. b+l-1 (clipped).  This fixes
    # the one-row/one-column asymmetry of even window sizes.
    H, W = 40, 37
    o, u, l, r = oracle.extents(h, w)
    for (a, b) in [(20, 18), (0, 0), (39, 36), (1, 35)]:
        I = np.zeros((H, W), np.uint8)
        I[a, b] = 1
        S1, _ = oracle.sums_recursive(I, h, w)
        exp = np.zeros((H, W), np.uint64)
        exp[max(a - u, 0):min(a + o - 1, H - 1) + 1, max(b - r, 0):min(b + l - 1, W - 1) + 1] = 1
        assert np.array_equal(S1.astype(np.uint64), exp)


def test_random_images_all_implementations_agree():
    for (H, W, h, w, seed) in [(150, 203, 75, 75, 1), (97, 301, 15, 151, 2), (64, 64, 151, 32, 3),
                               (33, 257, 257, 257, 4), (200, 50, 32, 31, 5)]:
        I = gen_document(H, W, seed, noise=10.0, stain=True)
        d1, d2 = oracle.sums_direct(I, h, w)
        r1, r2 = oracle.sums_recursive(I, h, w)
        i1, i2 = oracle.sums_integral(I, h, w)
        assert np.array_equal(d1, r1.astype(np.uint64)) and np.array_equal(d2, r2.astype(np.uint64))
        assert np.array_equal(d1, i1) and np.array_equal(d2, i2)


def test_strided_input_view():
    base = _rand(50, 80, 3)
    I = base[5:45, 7:70]  # row stride 80 > width 63
    a = oracle.sums_recursive(I, 9, 12)
    b = oracle.sums_recursive(np.ascontiguousarray(I), 9, 12)
    c = brute.sums_shift(np.ascontiguousarray(I), 9, 12)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0].astype(np.int64), c[0])
    ii = np.array([0, 39, 17, 3])
    jj = np.array([0, 62, 30, 61])
    s1, s2 = oracle.sums_direct_at(I, 9, 12, ii, jj)
    assert np.array_equal(s1.astype(np.int64), c[0][ii, jj])
    assert np.array_equal(s2.astype(np.int64), c[1][ii, jj])


def test_constant_image_and_bounds():
    for c in (0, 1, 137, 255):
        I = np.full((30, 45), c, np.uint8)
        n = oracle.count_map(30, 45, 11, 20)
        S1, S2 = oracle.sums_recursive(I, 11, 20)
        assert np.array_equal(S1.astype(np.int64), c * n)
        assert np.array_equal(S2.astype(np.int64), c * c * n)
    I = _rand(60, 70, 9)
    S1, S2 = oracle.sums_integral(I, 13, 21)
    n = oracle.count_map(60, 70, 13, 21)
    assert np.all(S1.astype(np.int64) <= 255 * n)
    assert np.all(S2.astype(np.int64) <= 65025 * n)


def test_linearity():
    A = _rand(40, 50, 1, hi=128)
    B = _rand(40, 50, 2, hi=128)
    a, _ = oracle.sums_recursive(A, 7, 10)
    b, _ = oracle.sums_recursive(B, 7, 10)
    c, _ = oracle.sums_recursive(A + B, 7, 10)
    assert np.array_equal(a.astype(np.int64) + b.astype(np.int64), c.astype(np.int64))


def test_total_sum_invariant():
    # sum_p S1(p) = sum_q I_q * N*(q), N*(q) = size of the reflected window.
    H, W, h, w = 45, 38, 10, 7
    I = _rand(H, W, 4)
    S1, _ = oracle.sums_recursive(I, h, w)
    o, u, l, r = oracle.extents(h, w)
    i = np.arange(H)
    j = np.arange(W)
    nr = np.minimum(i + o - 1, H - 1) - np.maximum(i - u, 0) + 1
    nc = np.minimum(j + l - 1, W - 1) - np.maximum(j - r, 0) + 1
    Nstar = nr[:, None] * nc[None, :]
    assert int(S1.astype(np.int64).sum()) == int((I.astype(np.int64) * Nstar).sum())


def test_paper_integer_ranges():
    # Section 3.3's accumulator widths: the extreme image (all 255) with the
    # largest window (257 x 257) keeps the 16-bit column sums and the 32-bit
    # window sum of squares exact.
    # the values Section 3.3 prints (tests/golden/paper_integer_ranges.txt)
    facts = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_integer_ranges.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, val = line.split("=")
                facts[key.strip()] = val.strip()
    assert 255 * 257 == int(facts["255*257"]) == 65535
    assert 255 * 255 * 257 == int(facts["255*255*257"]) < 2 ** 32 - 1
    assert int(facts["a4_600dpi"]) > 2 ** 32 / 255
    assert facts["2^32/255"].startswith("%.4f" % (2 ** 32 / 255))
    # the A4 page at 600 DPI: 8.27 x 11.7 inches
    assert int(facts["a4_600dpi"]) == round(8.27 * 600) * round(11.7 * 600)
    assert 65025 * 257 * 257 < 2 ** 32
    I = np.full((300, 300), 255, np.uint8)
    r1, r2 = oracle.sums_recursive(I, 257, 257)
    d1, d2 = oracle.sums_integral(I, 257, 257)
    assert np.array_equal(r1.astype(np.uint64), d1) and np.array_equal(r2.astype(np.uint64), d2)
    assert int(r2.max()) == 65025 * 257 * 257
    with pytest.raises(ValueError):
        oracle.sums_recursive(I, 258, 3)
