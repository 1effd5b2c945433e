"""Pins of the oracle's remaining Table 1 methods (Wolf, Feng, Rais,
Khurshid/NICK, Phansalkar) and of the global statistics L, M, S they use:
NumPy's own statistics, each method's formula evaluated in another algebraic
form from brute-force window sums, and the special cases where a method
reduces to Sauvola or to the window mean; and of Bernsen's midrange rule on
the window extremes, by brute force over clipped windows."""
import numpy as np
import pytest

import oracle
from docgen import gen_document

PARAMS = {
    oracle.WOLF: (0.5, 128.0),
    oracle.FENG: (0.9, 0.2, 0.3, 0.5, 128.0),
    oracle.RAIS: (),
    oracle.NICK: (-0.1,),
    oracle.PHANSALKAR: (2.0, 0.04, 0.25, 128.0),
}


def brute_moments(I, h, w):
    """Window S1, S2 and count n by direct summation over clipped windows,
    then m and s (population) in float64."""
    H, W = I.shape
    o, u, l, r = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    x = I.astype(np.float64)
    S1 = np.zeros((H, W))
    S2 = np.zeros((H, W))
    n = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            blk = x[max(i - o + 1, 0):min(i + u, H - 1) + 1, max(j - l + 1, 0):min(j + r, W - 1) + 1]
            S1[i, j] = blk.sum()
            S2[i, j] = (blk * blk).sum()
            n[i, j] = blk.size
    m = S1 / n
    s = np.sqrt(np.maximum(S2 / n - m * m, 0.0))
    return m, s, n, S2


def other_form(method, p, m, s, n, S2, L, M, S):
    """Each threshold in an algebraically equal form that shares no
    evaluation order with the oracle's sequence."""
    if method == oracle.WOLF:
        k, R = p
        return (1.0 - k) * m + k * L + k * (s / R) * (m - L)
    if method == oracle.FENG:
        a1, k1, k2, g, R = p
        x = s / R
        return a1 * m + (m - L) * k1 * np.power(x, 1.0 + g) + L * k2 * np.power(x, g)
    if method == oracle.RAIS:
        a, b = m * s, M * S
        e = np.maximum(a, b)
        f = np.divide(a - b, e, out=np.zeros_like(a), where=e > 0)
        return m + 0.3 * s * f
    if method == oracle.NICK:
        (k,) = p
        # Khurshid's own form: k times sqrt((sum of squares - m^2) / NP)
        return m + k * np.sqrt((S2 - m * m) / n)
    if method == oracle.PHANSALKAR:
        pp, q, k, R = p
        return m + m * pp * np.exp(-q * m) + m * k * (s / R - 1.0)
    raise ValueError(method)


def test_global_stats_match_numpy():
    for seed, (H, W) in enumerate([(1, 1), (7, 13), (120, 90)]):
        I = gen_document(H, W, 60 + seed, noise=10.0, stain=True)
        g = oracle.global_stats(I)
        assert g["L"] == I.min() and g["max"] == I.max()
        assert g["N"] == I.size
        assert g["T1"] == int(I.astype(np.int64).sum())
        assert g["T2"] == int((I.astype(np.int64) ** 2).sum())
        assert g["M"] == pytest.approx(float(I.astype(np.float64).mean()), rel=1e-14)
        assert g["S"] == pytest.approx(float(I.astype(np.float64).std()), rel=1e-12, abs=1e-12)


def test_global_stats_constant_image_has_zero_deviation():
    I = np.full((9, 11), 77, np.uint8)
    g = oracle.global_stats(I)
    assert g["S"] == 0.0 and g["M"] == 77.0 and g["L"] == 77.0


@pytest.mark.parametrize("method", sorted(PARAMS))
@pytest.mark.parametrize("H,W,h,w", [(23, 31, 7, 9), (16, 12, 15, 16), (9, 40, 4, 3)])
def test_table1_against_brute_force_in_another_form(method, H, W, h, w):
    I = gen_document(H, W, 70 + H, noise=10.0, stain=True)
    r = oracle.table1(I, h, w, method, PARAMS[method])
    g = r["gstats"]
    m, s, n, S2 = brute_moments(I, h, w)
    t2 = other_form(method, PARAMS[method], m, s, n, S2, g["L"], g["M"], g["S"])
    scale = np.maximum(np.abs(t2), 1.0)
    assert np.max(np.abs(r["t"] - t2) / scale) < 1e-9
    # masks agree wherever the threshold is not within rounding of the pixel
    clear = np.abs(I.astype(np.float64) - t2) > 1e-7 * scale
    assert np.array_equal(r["mask"][clear], (I.astype(np.float64) < t2)[clear].astype(np.uint8))


def test_wolf_with_zero_minimum_is_sauvola():
    # L = 0 turns m - k (m - L)(1 - s/R) into m (1 + k (s/R - 1))
    I = gen_document(50, 60, 5, noise=10.0, stain=True)
    I[0, 0] = 0
    k, R = 0.5, 128.0
    w = oracle.table1(I, 11, 11, oracle.WOLF, (k, R))
    sv = oracle.sauvola(I, 11, 11, k=k, R=R)
    assert np.max(np.abs(w["t"] - sv["t"]) / np.maximum(sv["t"], 1.0)) < 1e-13


def test_phansalkar_without_exponential_term_is_sauvola():
    I = gen_document(40, 70, 6, noise=10.0, stain=True)
    ph = oracle.table1(I, 9, 13, oracle.PHANSALKAR, (0.0, 0.04, 0.5, 128.0))
    sv = oracle.sauvola(I, 9, 13, k=0.5, R=128.0)
    assert np.array_equal(ph["t"], sv["t"])


def test_feng_reduces_to_the_window_mean():
    I = gen_document(30, 30, 7, noise=10.0)
    r = oracle.table1(I, 5, 7, oracle.FENG, (1.0, 0.0, 0.0, 0.7, 128.0))
    assert np.array_equal(r["t"], r["m"])


def test_rais_on_constant_image_is_the_mean():
    # every product m s and M S is 0: the fraction is taken as 0, t = m
    I = np.full((12, 15), 90, np.uint8)
    r = oracle.table1(I, 5, 5, oracle.RAIS, ())
    assert np.all(r["t"] == 90.0) and np.all(r["mask"] == 0)


def test_rais_offset_is_bounded_by_three_tenths_of_s():
    I = gen_document(40, 50, 8, noise=20.0, stain=True)
    r = oracle.table1(I, 9, 9, oracle.RAIS, ())
    assert np.all(np.abs(r["t"] - r["m"]) <= 0.3 * r["s"] * (1 + 1e-12) + 1e-12)


def test_nick_closed_form_on_constant_image():
    # s = 0: t = m + k m sqrt((n - 1)/n), n the clipped count
    I = np.full((6, 8), 200, np.uint8)
    h, w, k = 3, 5, -0.2
    r = oracle.table1(I, h, w, oracle.NICK, (k,))
    for (i, j) in [(0, 0), (2, 3), (5, 7)]:
        n = oracle.count_map(6, 8, h, w)[i, j]
        assert r["t"][i, j] == pytest.approx(200.0 + k * 200.0 * np.sqrt((n - 1) / n), rel=1e-15)


def test_table1_t_scalar_matches_image_routine():
    I = gen_document(20, 25, 9, noise=10.0, stain=True)
    for method, p in PARAMS.items():
        r = oracle.table1(I, 7, 7, method, p)
        g = r["gstats"]
        n = oracle.count_map(20, 25, 7, 7)
        for (i, j) in [(0, 0), (10, 12), (19, 24)]:
            t = oracle.table1_t(method, r["m"][i, j], r["s"][i, j], float(n[i, j]), p, g["L"], g["M"], g["S"])
            assert t == r["t"][i, j]


def test_bernsen_brute_force():
    # tiny images: the window extremes by explicit loops over clipped windows
    rng = np.random.default_rng(5)
    for (H, W, h, w, c) in [(7, 9, 3, 4, 15), (5, 5, 6, 2, 0), (11, 6, 5, 5, 100), (1, 8, 1, 3, 1)]:
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        o, u, l, r = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
        mask, mn, mx = oracle.bernsen(I, h, w, c)
        for i in range(H):
            for j in range(W):
                blk = I[max(i - o + 1, 0):min(i + u, H - 1) + 1, max(j - l + 1, 0):min(j + r, W - 1) + 1]
                lo, hi = int(blk.min()), int(blk.max())
                assert (mn[i, j], mx[i, j]) == (lo, hi)
                want = 1 if (hi - lo >= c and I[i, j] < (lo + hi) / 2) else 0
                assert mask[i, j] == want


def test_bernsen_low_contrast_windows_are_background():
    I = np.full((20, 30), 120, np.uint8)
    I[5:8, 10:13] = 126       # contrast 6 somewhere
    mask, mn, mx = oracle.bernsen(I, 7, 7, 7)
    assert not mask.any()
    mask, mn, mx = oracle.bernsen(I, 7, 7, 6)
    assert mask.any() and not mask[I == 126].any()
