"""Pins of the oracle's moments, Sauvola/Niblack thresholds and masks."""
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from docgen import gen_document

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split(None, 1)
        vals[key] = float(val)
    return vals


def test_checkerboard_golden():
    g = _golden("checkerboard_sauvola.txt")
    H, W, h, w = 40, 48, 8, 6
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    I = np.where((ii + jj) % 2 == 0, 0, 255).astype(np.uint8)
    res = oracle.sauvola(I, h, w, k=g["k"], R=g["R"])
    o, u, l, r = oracle.extents(h, w)
    inner = (slice(o - 1, H - u), slice(l - 1, W - r))  # windows fully inside
    assert np.all(res["m"][inner] == g["m"])
    assert np.all(res["s"][inner] == g["s"])
    assert np.all(res["t"][inner] == g["t"])
    assert np.array_equal(res["mask"][inner], (I[inner] == 0).astype(np.uint8))


@pytest.mark.parametrize("c", [0, 1, 100, 254, 255])
def test_constant_image(c):
    I = np.full((33, 47), c, np.uint8)
    for k in (0.0, 0.2, 0.5, 1.0):
        res = oracle.sauvola(I, 15, 9, k=k, R=128.0)
        assert np.all(res["s"] == 0.0)
        assert np.all(res["m"] == c)
        assert np.all(res["t"] == c * (1.0 - float(np.float32(k))))
        # t = c (1 - k) <= c, so the strict mask I < t is never set
        assert not res["mask"].any()
    nb = oracle.niblack(I, 15, 9, k=-0.2)
    assert np.all(nb["t"] == c) and not nb["mask"].any()


def test_popoviciu_bound_and_library_moments():
    I = gen_document(120, 160, 3, noise=10, stain=True)
    res = oracle.sauvola(I, 21, 17, k=0.5, R=128.0)
    assert res["s"].max() <= 127.5
    o, u, l, r = oracle.extents(21, 17)
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j = int(rng.integers(0, 120)), int(rng.integers(0, 160))
        win = I[max(i - o + 1, 0):i + u + 1, max(j - l + 1, 0):j + r + 1].astype(np.float64)
        assert res["m"][i, j] == pytest.approx(win.mean(), rel=1e-13)
        assert res["s"][i, j] == pytest.approx(win.std(ddof=0), rel=1e-9, abs=1e-9)


def test_extreme_variance_windows():
    # windows holding only 0 and 255 in equal numbers reach s = 127.5
    I = np.zeros((10, 10), np.uint8)
    I[:, 5:] = 255
    res = oracle.sauvola(I, 4, 10, k=0.5, R=128.0)
    assert res["s"][5, 4] == 127.5 and res["m"][5, 4] == 127.5  # columns 0..9


def test_shift_invariance_of_variance():
    I = gen_document(64, 80, 5, noise=10).astype(np.int32)
    I = np.clip(I, 0, 200).astype(np.uint8)
    a = oracle.sauvola(I, 9, 13)
    b = oracle.sauvola((I + 55).astype(np.uint8), 9, 13)
    n = oracle.count_map(64, 80, 9, 13)
    Va = n * a["S2"].astype(np.int64) - a["S1"].astype(np.int64) ** 2
    Vb = n * b["S2"].astype(np.int64) - b["S1"].astype(np.int64) ** 2
    assert np.array_equal(Va, Vb)
    assert np.all(Va >= 0)


def _exact_agreement(I, h, w, method, k, R=128.0):
    res = oracle.threshold(I, h, w, method, k, R)
    n = oracle.count_map(*I.shape, h, w)
    near = 0
    for (i, j), v in np.ndenumerate(I):
        args = (int(v), int(res["S1"][i, j]), int(res["S2"][i, j]), int(n[i, j]))
        if method == oracle.SAUVOLA:
            ex = brute.exact_below_sauvola(*args, k, R)
        else:
            ex = brute.exact_below_niblack(*args, k)
        if abs(float(v) - res["t"][i, j]) < 1e-9:
            near += 1
            continue
        assert bool(res["mask"][i, j]) == ex, (i, j)
    return near


def test_canonical_mask_matches_exact_rational_decision():
    # Away from exact ties the binary64 sequence decides every pixel as the
    # exact rational comparison does.
    I = gen_document(48, 56, 8, noise=10, stain=True)
    for (h, w, k) in [(7, 7, 0.5), (8, 5, 0.2), (15, 15, 0.34)]:
        _exact_agreement(I, h, w, oracle.SAUVOLA, k)
    for (h, w, k) in [(7, 9, -0.2), (6, 6, 0.3)]:
        _exact_agreement(I, h, w, oracle.NIBLACK, k)


def test_exact_ties_resolved_strictly():
    # constant windows give t = c exactly for k = 0: an exact tie, mask 0;
    # the exact decision agrees.
    I = np.full((8, 8), 90, np.uint8)
    res = oracle.sauvola(I, 3, 3, k=0.0)
    assert not res["mask"].any()
    assert not brute.exact_below_sauvola(90, 90 * 9, 8100 * 9, 9, 0.0, 128.0)


def test_sqrt_free_decision_agrees_away_from_ties():
    # Section 3.2: for k >= 0, I <= t iff I + m(k-1) <= 0 or
    # (I + m(k-1))^2 <= k^2 m^2 v / R^2; the paper's output is 1 - mask except at
    # exact ties.
    I = gen_document(96, 128, 4, noise=10, stain=True)
    for (h, w, k) in [(15, 15, 0.5), (32, 32, 0.2), (8, 31, 0.0)]:
        res = oracle.sauvola(I, h, w, k=k)
        pap = oracle.sauvola_sqrtfree(I, h, w, k, 128.0)
        far = np.abs(I.astype(np.float64) - res["t"]) > 1e-9
        assert np.array_equal(pap[far], 1 - res["mask"][far])


def test_k_zero_is_mean_threshold_and_niblack_equivalence():
    I = gen_document(64, 64, 6, noise=10)
    s0 = oracle.sauvola(I, 11, 11, k=0.0)
    n0 = oracle.niblack(I, 11, 11, k=0.0)
    assert np.array_equal(s0["t"], s0["m"])
    assert np.array_equal(s0["mask"], n0["mask"])


def test_large_R_limit():
    I = gen_document(40, 40, 7, noise=10)
    res = oracle.sauvola(I, 9, 9, k=0.4, R=1e30)
    assert np.allclose(res["t"], res["m"] * (1 - np.float64(np.float32(0.4))), rtol=1e-12)


def test_niblack_negative_k_exact():
    I = gen_document(30, 30, 9, noise=10)
    _exact_agreement(I, 5, 5, oracle.NIBLACK, -0.2)
    res = oracle.niblack(I, 5, 5, k=-0.2)
    assert np.allclose(res["t"], res["m"] - np.float64(np.float32(0.2)) * res["s"], rtol=1e-12)


@pytest.mark.parametrize("h,w,threads", [(75, 75, 7), (15, 9, 16), (32, 4, 3), (151, 31, 5), (4, 4, 40)])
def test_banded_runs_equal_the_whole_image(h, w, threads):
    # the CPU baseline runs the oracle on row bands with their halo rows on a
    # thread pool; its masks must equal the whole-image call
    I = gen_document(300, 257, 11, noise=10, stain=True)
    whole = oracle.sauvola(I, h, w, k=0.5, R=128.0)["mask"]
    assert np.array_equal(oracle.sauvola_bands(I, h, w, 0.5, 128.0, threads), whole)
