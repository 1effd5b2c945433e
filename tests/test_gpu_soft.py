"""GPU parity of the differentiable soft Sauvola: forward y and the gradients
with respect to I, k and R against the binary64 CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document, soft_batch

pytestmark = pytest.mark.gpu

TAU = 2.0
Y_ABS = 2e-5        # y tolerance (t within 1e-6 relative; sigmoid' <= 1/4, tau = 2)
GI_REL = 1e-4       # |gI - ref|_inf <= 1e-4 |ref|_inf
GKR_REL = 1e-5      # gk, gR relative
# gk and gR are sums over pixels of terms evaluated in float32 (sigmoid and
# products); their error is bounded by a few float32 units per term times the
# sum of the terms' magnitudes, which exceeds |sum| by orders of magnitude
# when the terms cancel.  Allowed: GKR_REL |ref| + GKR_COND sum|terms|.
GKR_COND = 1e-6


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def run(bz, I, k, R, h, w, g):
    It = torch.from_numpy(I).cuda().requires_grad_(True)
    kt = torch.from_numpy(np.asarray(k, np.float32)).cuda().requires_grad_(True)
    Rt = torch.tensor([R], dtype=torch.float32, device="cuda", requires_grad=True)
    y = bz.soft_sauvola(It, kt, Rt, h, w, TAU)
    (y * torch.from_numpy(g.astype(np.float32)).cuda()).sum().backward()
    return (y.detach().cpu().numpy(), It.grad.cpu().numpy(), kt.grad.cpu().numpy(),
            float(Rt.grad.cpu().numpy()[0]))


def compare(bz, I, k, R, h, w, g):
    y, gI, gk, gR = run(bz, I, k, R, h, w, g)
    ry, _ = oracle.soft_fwd(I, h, w, k, R, TAU)
    rgI, rgk, rgR = oracle.soft_bwd(I, g, h, w, k, R, TAU)
    assert np.max(np.abs(y - ry)) <= Y_ABS, np.max(np.abs(y - ry))
    assert np.max(np.abs(gI - rgI)) <= GI_REL * np.max(np.abs(rgI)), np.max(np.abs(gI - rgI)) / np.max(np.abs(rgI))
    assert np.allclose(gk, rgk, rtol=GKR_REL, atol=0), (gk, rgk)
    assert gR == pytest.approx(rgR, rel=GKR_REL)


# single-wave tiles (rows of at most 256 columns, aligned and ragged, up to
# the widest window they take) and four-wave tiles (wider rows or windows,
# one or several tiles per row); images shorter than the forward's 8-row
# strips and ragged last strips
@pytest.mark.parametrize("B,H,W,h,w", [(2, 64, 80, 7, 7), (3, 40, 33, 6, 9), (1, 100, 1500, 32, 32),
                                       (2, 300, 50, 75, 4), (1, 17, 19, 32, 32), (1, 1, 1, 3, 3),
                                       (1, 60, 256, 5, 129), (1, 60, 257, 5, 9), (1, 60, 200, 5, 130),
                                       (1, 90, 1100, 21, 75), (2, 70, 230, 9, 131), (1, 40, 1031, 3, 257),
                                       (2, 5, 70, 3, 3), (1, 13, 1030, 9, 5)])
def test_small_shapes(bz, B, H, W, h, w):
    I = np.stack([gen_document(H, W, 70 + b, noise=10, stain=True, dtype=np.float32) for b in range(B)])
    k = np.random.default_rng(B * H).uniform(0.2, 0.5, size=B).astype(np.float32)
    g = np.random.default_rng(W).standard_normal((B, H, W))
    compare(bz, I, k, 128.0, h, w, g)


def test_full_size_two_images(bz):
    # the 1024 x 1024 pages at h = w = 32 (each image is tiled exactly as in
    # the 32-image workload), full comparison for two images
    print("soft full size", flush=True)
    I, k, g = soft_batch(B=2)
    compare(bz, I, k, 128.0, 32, 32, g.astype(np.float64))


def _oracle_per_image(I, k, R, h, w, g, workers=8):
    """oracle.soft_fwd / soft_bwd image by image on a thread pool (the C
    oracle releases the GIL); the R gradient, a sum over every image and
    pixel, is the sum of the per-image sums.  Also the sums of the magnitudes
    of the k and R gradient terms: the same backward with |g| (with R above
    every window's s, each term of dL/dk and dL/dR has the sign of g)."""
    from concurrent.futures import ThreadPoolExecutor
    assert R > 127.5  # s <= 127.5 for values in [0, 255] (Popoviciu)

    def one(b):
        ry, _ = oracle.soft_fwd(I[b:b + 1], h, w, k[b:b + 1], R, TAU)
        rgI, rgk, rgR = oracle.soft_bwd(I[b:b + 1], g[b:b + 1], h, w, k[b:b + 1], R, TAU)
        _, agk, agR = oracle.soft_bwd(I[b:b + 1], np.abs(g[b:b + 1]), h, w, k[b:b + 1], R, TAU)
        return ry[0], rgI[0], rgk[0], rgR, agk[0], agR

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, range(I.shape[0])))
    ry = np.stack([r[0] for r in res])
    rgI = np.stack([r[1] for r in res])
    rgk = np.array([r[2] for r in res])
    rgR = float(np.sum([r[3] for r in res]))
    agk = np.array([r[4] for r in res])
    agR = float(np.sum([r[5] for r in res]))
    return ry, rgI, rgk, rgR, agk, agR


def test_batch_32_against_oracle(bz):
    # the 32-image workload (32 x 1024 x 1024, h = w = 32, k per image, one R):
    # y and gI of every image, gk of every image and gR summed over all 32,
    # against the binary64 oracle
    print("soft 32-image workload", flush=True)
    I, k, g = soft_batch(B=32)
    y, gI, gk, gR = run(bz, I, k, 128.0, 32, 32, g)
    ry, rgI, rgk, rgR, agk, agR = _oracle_per_image(I, k, 128.0, 32, 32, g.astype(np.float64))
    assert np.max(np.abs(y - ry)) <= Y_ABS, np.max(np.abs(y - ry))
    for b in range(I.shape[0]):
        ref = np.max(np.abs(rgI[b]))
        assert np.max(np.abs(gI[b] - rgI[b])) <= GI_REL * ref, (b, np.max(np.abs(gI[b] - rgI[b])) / ref)
    err = np.abs(gk - rgk)
    assert np.all(err <= GKR_REL * np.abs(rgk) + GKR_COND * agk), (err, rgk, agk)
    assert abs(gR - rgR) <= GKR_REL * abs(rgR) + GKR_COND * agR, (gR, rgR, agR)
    # images 0 and 1 of the batch give the bits of a batch of those two alone
    y2, gI2, gk2, _ = run(bz, I[:2], k[:2], 128.0, 32, 32, g[:2])
    assert np.array_equal(y[:2], y2) and np.array_equal(gI[:2], gI2) and np.array_equal(gk[:2], gk2)


def test_gradients_take_the_callers_shapes(bz):
    # k of shape (B, 1) and a 0-d R: the gradients come back in those shapes
    I = np.stack([gen_document(40, 48, 90 + b, noise=10, stain=True, dtype=np.float32) for b in range(2)])
    g = np.random.default_rng(5).standard_normal(I.shape)
    It = torch.from_numpy(I).cuda().requires_grad_(True)
    kt = torch.tensor([[0.3], [0.4]], dtype=torch.float32, device="cuda", requires_grad=True)
    Rt = torch.tensor(128.0, dtype=torch.float32, device="cuda", requires_grad=True)
    y = bz.soft_sauvola(It, kt, Rt, 7, 9, TAU)
    (y * torch.from_numpy(g.astype(np.float32)).cuda()).sum().backward()
    assert kt.grad.shape == (2, 1) and Rt.grad.shape == ()
    _, rgk, rgR = oracle.soft_bwd(I, g, 7, 9, np.array([0.3, 0.4], np.float32), 128.0, TAU)
    assert np.allclose(kt.grad.cpu().numpy()[:, 0], rgk, rtol=GKR_REL, atol=0)
    assert float(Rt.grad) == pytest.approx(rgR, rel=GKR_REL)
    # one 2-D image with a (1, 1) k
    I1 = torch.from_numpy(I[0]).cuda().requires_grad_(True)
    k1 = torch.tensor([[0.3]], dtype=torch.float32, device="cuda", requires_grad=True)
    y1 = bz.soft_sauvola(I1, k1, Rt, 7, 9, TAU)
    assert y1.shape == I1.shape
    y1.sum().backward()
    assert I1.grad.shape == I1.shape and k1.grad.shape == (1, 1)


@pytest.mark.parametrize("B,H,W,h,w", [(2, 1024, 1024, 32, 32), (1, 2000, 40, 31, 31), (1, 1024, 300, 257, 5)])
def test_running_sums_do_not_drift(bz, B, H, W, h, w):
    # the binary64 running sums of the soft kernels over full sweeps down
    # real-valued images agree with the direct binary64 window sums to 1e-12
    # relative (the add/subtract recurrence restarts with every strip)
    print("soft sums", B, H, W, h, w, flush=True)
    I = np.stack([gen_document(H, W, 300 + b, noise=10, stain=True, dtype=np.float32) for b in range(B)])
    S1, S2 = bz.soft_window_sums(torch.from_numpy(I).cuda(), h, w)
    S1, S2 = S1.cpu().numpy(), S2.cpu().numpy()
    for b in range(B):
        x = I[b].astype(np.float64)
        r1 = oracle.box_f64(x, h, w)
        r2 = oracle.box_f64(x * x, h, w)
        assert np.max(np.abs(S1[b] - r1) / r1) <= 1e-12, np.max(np.abs(S1[b] - r1) / r1)
        assert np.max(np.abs(S2[b] - r2) / r2) <= 1e-12, np.max(np.abs(S2[b] - r2) / r2)


def test_deterministic(bz):
    I, k, g = soft_batch(B=3, H=256, W=300)
    a = run(bz, I, k, 100.0, 15, 17, g)
    b = run(bz, I, k, 100.0, 15, 17, g)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_k_zero_R_gradient(bz):
    I = gen_document(50, 60, 3, noise=10, dtype=np.float32)[None]
    g = np.random.default_rng(1).standard_normal(I.shape)
    _, _, _, gR = run(bz, I, np.zeros(1, np.float32), 128.0, 9, 9, g)
    assert gR == 0.0


def test_tall_image_no_drift(bz):
    # 2000 rows: the binary64 running sums restart with every strip, so the
    # last rows match the oracle as well as the first
    I = gen_document(2000, 40, 17, noise=10, stain=True, dtype=np.float32)[None]
    k = np.array([0.35], np.float32)
    g = np.random.default_rng(17).standard_normal(I.shape)
    compare(bz, I, k, 128.0, 31, 31, g)


def test_strided_rows_match_contiguous(bz):
    # row stride ld = W + 3 (no 16-byte row loads) gives the bits of the
    # contiguous call
    import ctypes
    lib = bz.lib
    B, H, W, ld, h, w, tau = 2, 70, 96, 99, 9, 11, 2.0
    I = np.stack([gen_document(H, W, 40 + b, noise=10, stain=True, dtype=np.float32) for b in range(B)])
    g = np.random.default_rng(3).standard_normal((B, H, W)).astype(np.float32)
    k = torch.tensor([0.3, 0.45], dtype=torch.float32, device="cuda")
    R = torch.tensor([128.0], dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def padded(a):
        p = torch.zeros((B, H, ld), dtype=torch.float32, device="cuda")
        p[:, :, :W] = torch.from_numpy(a).cuda()
        return p

    def run_c(Ib, gb, stride):
        y = torch.full_like(Ib, -7.0)
        gI = torch.full_like(Ib, -7.0)
        gk = torch.empty(B, dtype=torch.float32, device="cuda")
        gR = torch.empty(1, dtype=torch.float32, device="cuda")
        nb = int(lib.bz_soft_workspace_size(B, H, W))
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        assert lib.bz_soft_sauvola_fwd(Ib.data_ptr(), B, H, W, stride, h, w, k.data_ptr(), R.data_ptr(), tau,
                                       y.data_ptr(), st) == 0
        assert lib.bz_soft_sauvola_bwd(Ib.data_ptr(), gb.data_ptr(), B, H, W, stride, h, w, k.data_ptr(),
                                       R.data_ptr(), tau, gI.data_ptr(), gk.data_ptr(), gR.data_ptr(),
                                       ws.data_ptr(), nb, st) == 0
        torch.cuda.synchronize()
        return y[:, :, :W].cpu().numpy(), gI[:, :, :W].cpu().numpy(), gk.cpu().numpy(), gR.cpu().numpy(), \
            y[:, :, W:].cpu().numpy(), gI[:, :, W:].cpu().numpy()

    a = run_c(torch.from_numpy(I).cuda(), torch.from_numpy(g).cuda(), W)
    b = run_c(padded(I), padded(g), ld)
    for x, z in zip(a[:4], b[:4]):
        assert np.array_equal(x, z)
    # the padding columns of the outputs are not written
    assert np.all(b[4] == -7.0) and np.all(b[5] == -7.0)


@pytest.mark.parametrize("fwd,bwd,adj", [(8, 8, 8), (17, 32, 8), (32, 8, 32), (11, 20, 13)])
def test_strip_overrides(bz, monkeypatch, fwd, bwd, adj):
    # the strips of each phase (tuning overrides, 8 to 32 rows) change only
    # the rounding of the binary64 running sums: every setting stays within
    # the tolerances of the oracle
    monkeypatch.setenv("BZ_SOFT_STRIP", str(fwd))
    monkeypatch.setenv("BZ_SOFT_STRIP_BWD", str(bwd))
    monkeypatch.setenv("BZ_SOFT_STRIP_ADJ", str(adj))
    B, H, W, h, w = 2, 100, 300, 21, 15
    I = np.stack([gen_document(H, W, 90 + b, noise=10, stain=True, dtype=np.float32) for b in range(B)])
    k = np.random.default_rng(7).uniform(0.2, 0.5, size=B).astype(np.float32)
    g = np.random.default_rng(8).standard_normal((B, H, W))
    compare(bz, I, k, 128.0, h, w, g)
