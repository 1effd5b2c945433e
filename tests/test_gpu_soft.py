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
# one or several tiles per row)
@pytest.mark.parametrize("B,H,W,h,w", [(2, 64, 80, 7, 7), (3, 40, 33, 6, 9), (1, 100, 1500, 32, 32),
                                       (2, 300, 50, 75, 4), (1, 17, 19, 32, 32), (1, 1, 1, 3, 3),
                                       (1, 60, 256, 5, 129), (1, 60, 257, 5, 9), (1, 60, 200, 5, 130),
                                       (1, 90, 1100, 21, 75), (2, 70, 230, 9, 131), (1, 40, 1031, 3, 257)])
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


def test_batch_32_matches_per_image(bz):
    # the 32-image workload: images 0 and 1 of the full batch give the same
    # y and gI as a batch of those two alone, and gk is per image
    I, k, g = soft_batch(B=32)
    y32, gI32, gk32, gR32 = run(bz, I, k, 128.0, 32, 32, g)
    y2, gI2, gk2, gR2 = run(bz, I[:2], k[:2], 128.0, 32, 32, g[:2])
    assert np.array_equal(y32[:2], y2) and np.array_equal(gI32[:2], gI2)
    assert np.array_equal(gk32[:2], gk2)
    assert np.isfinite(gR32) and np.all(np.isfinite(gk32))


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
