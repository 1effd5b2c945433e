"""Pins of the oracle's differentiable (soft) Sauvola forward and backward."""
import numpy as np
import pytest

import oracle
from docgen import gen_document

TAU = 2.0


def _crop(seed, H=24, W=20):
    return gen_document(H, W, seed, noise=10.0, stain=True, dtype=np.float32)


def test_adjoint_identity_exact_integers():
    # <B x, y> = <x, B* y> exactly for integer fields (all partial sums are
    # exact in binary64): pins the reflected window and its clipping.
    rng = np.random.default_rng(3)
    for (H, W, h, w) in [(13, 17, 4, 5), (20, 9, 7, 6), (8, 8, 12, 3), (16, 16, 1, 1)]:
        x = rng.integers(-50, 50, size=(H, W)).astype(np.float64)
        y = rng.integers(-50, 50, size=(H, W)).astype(np.float64)
        lhs = float(np.sum(oracle.box_f64(x, h, w) * y))
        rhs = float(np.sum(x * oracle.box_adjoint(y, h, w)))
        assert lhs == rhs


def test_adjoint_of_impulse_is_window_indicator():
    H, W, h, w = 15, 14, 6, 5
    o, u, l, r = oracle.extents(h, w)
    G = np.zeros((H, W))
    p = (7, 6)
    G[p] = 1.0
    out = oracle.box_adjoint(G, h, w)
    want = np.zeros((H, W))
    want[p[0] - o + 1:p[0] + u + 1, p[1] - l + 1:p[1] + r + 1] = 1.0
    assert np.array_equal(out, want)


def test_float_sums_match_integer_oracle():
    # On integer-valued float images the soft path's window moments equal the
    # integer oracle's (all sums exact).
    I8 = gen_document(30, 26, 4, noise=10)
    y, t = oracle.soft_fwd(I8.astype(np.float32), 7, 9, 0.5, 128.0, TAU)
    ref = oracle.sauvola(I8, 7, 9, k=0.5, R=128.0)
    assert np.allclose(t[0], ref["t"], rtol=1e-14, atol=1e-12)


def test_checkerboard_threshold_golden():
    H, W = 20, 24
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    I = np.where((ii + jj) % 2 == 0, 0.0, 255.0).astype(np.float32)
    y, t = oracle.soft_fwd(I, 6, 8, 0.5, 128.0, TAU)
    assert t[0, 10, 10] == 127.2509765625
    z = (255.0 - 127.2509765625) / TAU
    assert y[0, 10, 11 if (10 + 11) % 2 else 10] == pytest.approx(1 / (1 + np.exp(-z)), rel=1e-15)


def _loss(I, g, h, w, k, R):
    y, _ = oracle.soft_fwd(I, h, w, k, R, TAU)
    return float(np.sum(g * y))


@pytest.mark.parametrize("h,w", [(5, 5), (6, 4)])
def test_gradients_match_central_differences(h, w):
    B, H, W = 2, 18, 16
    I = np.stack([_crop(50 + b, H, W) for b in range(B)])
    g = np.random.default_rng(9).standard_normal((B, H, W))
    k = np.array([0.3, 0.45])
    R = 128.0
    gI, gk, gR = oracle.soft_bwd(I, g, h, w, k, R, TAU)
    rng = np.random.default_rng(1)
    pts = [(0, 0, 0), (1, H - 1, W - 1), (0, 0, W - 1), (1, H - 1, 0)]
    pts += [(int(rng.integers(B)), int(rng.integers(H)), int(rng.integers(W))) for _ in range(24)]
    # I is float32 data; the finite difference is taken in binary64 on a
    # float64 copy, so the oracle forward is evaluated through a float64 path.
    for (b, i, j) in pts:
        eps = 1e-3
        Ip = I.astype(np.float64)
        Im = I.astype(np.float64)
        Ip[b, i, j] += eps
        Im[b, i, j] -= eps
        fd = (_loss64(Ip, g, h, w, k, R) - _loss64(Im, g, h, w, k, R)) / (2 * eps)
        assert gI[b, i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    for b in range(B):
        eps = 1e-6
        kp = k.copy(); kp[b] += eps
        km = k.copy(); km[b] -= eps
        fd = (_loss64(I.astype(np.float64), g, h, w, kp, R) - _loss64(I.astype(np.float64), g, h, w, km, R)) / (2 * eps)
        assert gk[b] == pytest.approx(fd, rel=1e-6)
    eps = 1e-4
    fd = (_loss64(I.astype(np.float64), g, h, w, k, R + eps) - _loss64(I.astype(np.float64), g, h, w, k, R - eps)) / (2 * eps)
    assert gR == pytest.approx(fd, rel=1e-6)


def test_gradients_match_central_differences_on_64x64_crops():
    # 64 x 64 crops of the differentiable workload's pages, each crop an
    # image of its own, at the workload's window h = w = 32 (so most windows
    # are clipped); central differences in binary64 at every border pixel
    # and at 256 sampled interior pixels, and for every k and R, against the
    # oracle's analytic gradient to 1e-6 relative
    from docgen import soft_batch
    h = w = 32
    pages, kk, wr = soft_batch(B=2)
    rng = np.random.default_rng(64)
    offs = [(int(rng.integers(0, 1024 - 64)), int(rng.integers(0, 1024 - 64))) for _ in range(2)]
    I = np.stack([pages[b, i:i + 64, j:j + 64] for b, (i, j) in enumerate(offs)])
    g = np.stack([wr[b, i:i + 64, j:j + 64] for b, (i, j) in enumerate(offs)]).astype(np.float64)
    k = kk.astype(np.float64)
    R = 128.0
    B, H, W = I.shape
    gI, gk, gR = oracle.soft_bwd(I, g, h, w, k, R, TAU)
    border = [(i, j) for i in range(H) for j in range(W) if i in (0, H - 1) or j in (0, W - 1)]
    inner = [(int(rng.integers(1, H - 1)), int(rng.integers(1, W - 1))) for _ in range(256)]
    I64 = I.astype(np.float64)
    for b in range(B):
        one = lambda X, kb=k[b:b + 1], gb=g[b:b + 1], RR=R: _loss64(X[None], gb, h, w, kb, RR)
        for (i, j) in border + inner:
            eps = 1e-3
            Ip = I64[b].copy()
            Im = I64[b].copy()
            Ip[i, j] += eps
            Im[i, j] -= eps
            fd = (one(Ip) - one(Im)) / (2 * eps)
            assert gI[b, i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9), (b, i, j)
        eps = 1e-6
        fd = (_loss64(I64[b][None], g[b:b + 1], h, w, k[b:b + 1] + eps, R)
              - _loss64(I64[b][None], g[b:b + 1], h, w, k[b:b + 1] - eps, R)) / (2 * eps)
        assert gk[b] == pytest.approx(fd, rel=1e-6)
    eps = 1e-4
    fd = (_loss64(I64, g, h, w, k, R + eps) - _loss64(I64, g, h, w, k, R - eps)) / (2 * eps)
    assert gR == pytest.approx(fd, rel=1e-6)


def _loss64(I64, g, h, w, k, R):
    """Loss of a float64 image stack, evaluated with the plain NumPy form of
    the same forward (window sums from the integral images of Section 2)."""
    B, H, W = I64.shape
    o, u, l, r = oracle.extents(h, w)
    n = oracle.count_map(H, W, h, w).astype(np.float64)
    tot = 0.0
    for b in range(B):
        x = I64[b]
        J1 = np.zeros((H + 1, W + 1)); J1[1:, 1:] = x.cumsum(0).cumsum(1)
        J2 = np.zeros((H + 1, W + 1)); J2[1:, 1:] = (x * x).cumsum(0).cumsum(1)
        a0 = np.maximum(np.arange(H) - o, -1) + 1
        a1 = np.minimum(np.arange(H) + u, H - 1) + 1
        b0 = np.maximum(np.arange(W) - l, -1) + 1
        b1 = np.minimum(np.arange(W) + r, W - 1) + 1
        S1 = J1[a1][:, b1] - J1[a0][:, b1] - J1[a1][:, b0] + J1[a0][:, b0]
        S2 = J2[a1][:, b1] - J2[a0][:, b1] - J2[a1][:, b0] + J2[a0][:, b0]
        m = S1 / n
        v = np.maximum((n * S2 - S1 * S1) / (n * n), 0.0)
        s = np.sqrt(v)
        t = m * (1 + k[b] * (s / R - 1))
        y = 1 / (1 + np.exp(-(x - t) / TAU))
        tot += float(np.sum(g[b] * y))
    return tot


def test_numpy_forward_matches_oracle_forward():
    I = np.stack([_crop(60), _crop(61)])
    k = np.array([0.2, 0.5])
    g = np.ones_like(I, dtype=np.float64)
    y, _ = oracle.soft_fwd(I, 7, 6, k, 128.0, TAU)
    assert _loss64(I.astype(np.float64), g, 7, 6, k, 128.0) == pytest.approx(float(y.sum()), rel=1e-13)


def test_k_zero_gives_zero_R_gradient():
    I = _crop(70)[None]
    g = np.random.default_rng(2).standard_normal(I.shape)
    _, _, gR = oracle.soft_bwd(I, g, 5, 5, np.array([0.0]), 128.0, TAU)
    assert gR == 0.0


def test_small_tau_limit_is_paper_polarity():
    # y -> 1 where I > t (the paper's output bit), i.e. 1 - mask away from ties
    I8 = gen_document(30, 30, 12, noise=10)
    y, t = oracle.soft_fwd(I8.astype(np.float32), 9, 9, 0.4, 128.0, 1e-3)
    ref = oracle.sauvola(I8, 9, 9, k=0.4)
    far = np.abs(I8 - ref["t"]) > 0.05
    assert np.array_equal((y[0][far] > 0.5).astype(np.uint8), 1 - ref["mask"][far])
