"""GPU parity of the window sums, moments and Sauvola/Niblack masks against
the CPU oracle (bit-exact integers and masks; m, s within 1e-6 relative)."""
import os

import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document

pytestmark = pytest.mark.gpu

REL = 1e-6  # m, s tolerance against binary64


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def log(*a):
    print(*a, flush=True)


def check_sums(bz, I, h, w, ref=None):
    S1, S2 = bz.window_sums(dev(I), h, w)
    torch.cuda.synchronize()
    if ref is None:
        ref = oracle.sums_recursive(I, h, w)
    assert np.array_equal(u32(S1), ref[0]), ("S1", I.shape, h, w)
    assert np.array_equal(u32(S2), ref[1]), ("S2", I.shape, h, w)


def test_sums_small_document(bz):
    I = gen_document(384, 512, 1)
    log("sums 384x512 h=w=32")
    check_sums(bz, I, 32, 32)


def test_sums_exhaustive_tiny(bz):
    rng = np.random.default_rng(11)
    log("exhaustive tiny sweep")
    for H in range(1, 13):
        for W in range(1, 13):
            I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
            d = dev(I)
            for h in range(1, 10):
                for w in range(1, 10):
                    S1, S2 = bz.window_sums(d, h, w)
                    r1, r2 = oracle.sums_recursive(I, h, w)
                    assert np.array_equal(u32(S1), r1), (H, W, h, w)
                    assert np.array_equal(u32(S2), r2), (H, W, h, w)


@pytest.mark.parametrize("H,W,h,w", [(257, 300, 257, 257), (100, 4096, 151, 151), (70, 5000, 151, 75),
                                     (90, 9001, 32, 257), (33, 4100, 2, 2), (1, 4097, 5, 4),
                                     (777, 1, 75, 3), (300, 1025, 64, 63)])
def test_sums_shapes_and_column_tiles(bz, H, W, h, w):
    log("sums", H, W, h, w)
    I = gen_document(H, W, H + W, noise=10, stain=True)
    check_sums(bz, I, h, w)


def test_sums_extreme_values(bz):
    I = np.full((300, 280), 255, np.uint8)
    check_sums(bz, I, 257, 257)
    check_sums(bz, np.zeros((50, 60), np.uint8), 9, 9)


@pytest.mark.parametrize("off,ld", [(1, 515), (3, 512), (0, 513), (2, 1030)])
def test_sums_unaligned_strided(bz, off, ld):
    # base pointer offsets and row strides that rule out dword access
    H, W = 200, 500
    buf = np.random.default_rng(off).integers(0, 256, size=(H * ld + off + 8,), dtype=np.uint8)
    d = dev(buf)
    view = d[off:off + H * ld].view(H, ld)[:, :W]
    host = buf[off:off + H * ld].reshape(H, ld)[:, :W]
    S1, S2 = bz.window_sums(view, 17, 24)
    r1, r2 = oracle.sums_recursive(np.ascontiguousarray(host), 17, 24)
    assert np.array_equal(u32(S1), r1) and np.array_equal(u32(S2), r2)


@pytest.mark.parametrize("off,W", [(0, 497), (1, 498), (2, 499), (3, 501), (1, 7), (2, 2)])
def test_unaligned_width_tight_rows(bz, off, W):
    # widths that are not multiples of 4, rows packed at a stride of W and a
    # shifted base: every row starts at a different misalignment, the last
    # lane of a row holds fewer than four columns, and the image ends at the
    # end of its buffer
    H = 150
    buf = np.random.default_rng(W).integers(0, 256, size=(H * W + off,), dtype=np.uint8)
    d = dev(buf)
    view = d[off:].view(H, W)
    host = buf[off:].reshape(H, W)
    for h, w in ((17, 24), (1, 3), (31, 9)):
        S1, S2 = bz.window_sums(view, h, w)
        r1, r2 = oracle.sums_recursive(np.ascontiguousarray(host), h, w)
        assert np.array_equal(u32(S1), r1) and np.array_equal(u32(S2), r2), (off, W, h, w)
    mask, m, s = bz.sauvola(view, 15, 15, k=0.5, R=128.0)
    ref = oracle.sauvola(np.ascontiguousarray(host), 15, 15, k=0.5, R=128.0)
    assert mask_report(mask.cpu().numpy(), ref, host) == 0


def check_moments(m, s, ref, S1, S2, n):
    m = m.cpu().numpy().astype(np.float64)
    s = s.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(m - ref["m"]) <= REL * np.abs(ref["m"])), np.max(np.abs(m - ref["m"]) / np.maximum(ref["m"], 1e-300))
    assert np.all(np.abs(s - ref["s"]) <= REL * np.abs(ref["s"]))
    Vn = n * S2.astype(np.int64) - S1.astype(np.int64) ** 2
    assert np.array_equal(s == 0, Vn == 0)


def mask_report(got, ref, I):
    bad = got != ref["mask"]
    nbad = int(bad.sum())
    near = int((np.abs(I.astype(np.float64) - ref["t"]) < 1e-4).sum())
    log("mask disagreements", nbad, "oracle near-ties", near)
    return nbad


@pytest.mark.parametrize("h", [32, 7, 8])
def test_mean_std_small(bz, h):
    I = gen_document(384, 512, 1)
    m, s = bz.window_mean_std(dev(I), h, h + 1)
    ref = oracle.sauvola(I, h, h + 1)
    n = oracle.count_map(384, 512, h, h + 1)
    check_moments(m, s, ref, ref["S1"], ref["S2"], n)


def test_sauvola_config0(bz):
    I = gen_document(384, 512, 1)
    mask, m, s = bz.sauvola(dev(I), 32, 32, k=0.5, R=128.0)
    ref = oracle.sauvola(I, 32, 32, k=0.5, R=128.0)
    assert mask_report(mask.cpu().numpy(), ref, I) == 0
    check_moments(m, s, ref, ref["S1"], ref["S2"], oracle.count_map(384, 512, 32, 32))


@pytest.mark.parametrize("win", [15, 32, 75, 151])
@pytest.mark.parametrize("method", ["sauvola", "niblack"])
def test_full_size_masks_and_moments(bz, win, method):
    # the 4096 x 3072 page of the headline workload, every window size
    log("full size", method, win)
    I = _page()
    if method == "sauvola":
        mask, m, s = bz.sauvola(dev(I), win, win, k=0.5, R=128.0)
        ref = oracle.sauvola(I, win, win, k=0.5, R=128.0)
    else:
        mask, m, s = bz.niblack(dev(I), win, win, k=-0.2)
        ref = oracle.niblack(I, win, win, k=-0.2)
    assert mask_report(mask.cpu().numpy(), ref, I) == 0
    check_moments(m, s, ref, ref["S1"], ref["S2"], oracle.count_map(*I.shape, win, win))


_PAGE = {}


def _page():
    if "p" not in _PAGE:
        _PAGE["p"] = gen_document(3072, 4096, 2, noise=10.0, stain=True)
    return _PAGE["p"]


def test_full_size_sums_exact(bz):
    I = _page()
    for win in (15, 151):
        log("full size sums", win)
        check_sums(bz, I, win, win)


def test_reference_sequence_bit_exact_everywhere(bz, monkeypatch):
    # Decide EVERY pixel with the device's binary64 sequence (division, square
    # root, multiply-adds with contraction off) and compare with the CPU's.
    monkeypatch.setenv("BZ_FORCE_REFERENCE", "1")
    I = gen_document(1024, 1536, 21, noise=10.0, stain=True)
    for (h, w, k) in [(31, 31, 0.5), (16, 9, 0.2), (75, 75, 0.34)]:
        mask, _, _ = bz.sauvola(dev(I), h, w, k=k, R=128.0, stats=False)
        ref = oracle.sauvola(I, h, w, k=k, R=128.0)
        assert mask_report(mask.cpu().numpy(), ref, I) == 0
    for (h, w, k) in [(15, 15, -0.2), (40, 41, 0.7)]:
        mask, _, _ = bz.niblack(dev(I), h, w, k=k, stats=False)
        ref = oracle.niblack(I, h, w, k=k)
        assert mask_report(mask.cpu().numpy(), ref, I) == 0


def test_ties_and_degenerate_images(bz):
    # constant pages (s = 0, t = c(1-k)), the 0/255 checkerboard (s = 127.5),
    # k = 0 (t = m exactly: many exact ties with constant windows), tiny images
    cases = [np.full((64, 80), 0, np.uint8), np.full((64, 80), 255, np.uint8),
             np.full((5, 3), 17, np.uint8)]
    ii, jj = np.meshgrid(np.arange(64), np.arange(72), indexing="ij")
    cases.append(np.where((ii + jj) % 2 == 0, 0, 255).astype(np.uint8))
    rng = np.random.default_rng(4)
    blocky = np.kron(rng.integers(0, 4, size=(16, 16)) * 60, np.ones((8, 8))).astype(np.uint8)
    cases.append(blocky)
    for I in cases:
        for (h, w, k) in [(8, 6, 0.5), (3, 3, 0.0), (1, 1, 0.2), (16, 16, 0.0)]:
            mask, _, _ = bz.sauvola(dev(I), h, w, k=k, R=128.0)
            ref = oracle.sauvola(I, h, w, k=k, R=128.0)
            assert mask_report(mask.cpu().numpy(), ref, I) == 0, (I.shape, h, w, k)
            mask, _, _ = bz.niblack(dev(I), h, w, k=-k)
            ref = oracle.niblack(I, h, w, k=-k)
            assert mask_report(mask.cpu().numpy(), ref, I) == 0, (I.shape, h, w, -k)


@pytest.mark.parametrize("H,W,win", [(333, 4097, 75), (64, 9000, 151), (5, 5, 32), (1000, 123, 15)])
def test_mask_shapes_and_tiles(bz, H, W, win):
    I = gen_document(H, W, 7 * H + W, noise=10.0, stain=True)
    mask, m, s = bz.sauvola(dev(I), win, win, k=0.3, R=100.0)
    ref = oracle.sauvola(I, win, win, k=0.3, R=100.0)
    assert mask_report(mask.cpu().numpy(), ref, I) == 0
    check_moments(m, s, ref, ref["S1"], ref["S2"], oracle.count_map(H, W, win, win))


def test_mask_only_and_strided_outputs(bz):
    I = gen_document(300, 640, 5, noise=10.0)
    d = dev(I)
    mask, m, s = bz.sauvola(d, 21, 21, stats=False)
    assert m is None and s is None
    ref = oracle.sauvola(I, 21, 21)
    assert mask_report(mask.cpu().numpy(), ref, I) == 0
    big = torch.zeros((300, 700), dtype=torch.uint8, device="cuda")
    bm = torch.zeros((300, 650), dtype=torch.float32, device="cuda")
    bs = torch.zeros((300, 650), dtype=torch.float32, device="cuda")
    bz.sauvola(d, 21, 21, mask=big[:, 3:643], mean=bm[:, 1:641], std=bs[:, 1:641])
    assert mask_report(big[:, 3:643].cpu().numpy(), ref, I) == 0
    assert np.all(big[:, :3].cpu().numpy() == 0) and np.all(big[:, 643:].cpu().numpy() == 0)
    check_moments(bm[:, 1:641], bs[:, 1:641], ref, ref["S1"], ref["S2"], oracle.count_map(300, 640, 21, 21))


def test_given_outputs_are_checked(bz):
    # outputs the caller passes must match the image: shape, dtype, device and
    # unit column stride, and mean/std one row stride; a given mean with a
    # padded stride gets a std of the same stride
    d = dev(gen_document(40, 50, 6, noise=10.0))
    u8 = lambda *s: torch.zeros(s, dtype=torch.uint8, device="cuda")
    f32 = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    bad = [dict(mask=u8(40, 49)), dict(mask=u8(50, 40).t()),
           dict(mask=torch.zeros((40, 50), dtype=torch.int32, device="cuda")),
           dict(mask=torch.zeros((40, 50), dtype=torch.uint8)),
           dict(mean=f32(40, 50).double()), dict(mean=f32(50, 40).t()),
           dict(mean=f32(40, 50), std=f32(40, 60)[:, :50])]
    for kw in bad:
        with pytest.raises(ValueError):
            bz.sauvola(d, 7, 7, **kw)
    with pytest.raises(ValueError):
        bz.sauvola(d, 7, 7, stats=False, mean=f32(40, 50))
    m0, s0 = bz.sauvola(d, 7, 7)[1:]
    wide = f32(40, 64)
    _, m, s = bz.sauvola(d, 7, 7, mean=wide[:, :50])
    assert s.stride(0) == 64 and torch.equal(m, m0) and torch.equal(s, s0)


@pytest.mark.parametrize("strip,threads", [(1, 0), (3, 0), (50, 128), (7, 64), (0, 192)])
def test_tiling_overrides(bz, monkeypatch, strip, threads):
    # other strip heights and block sizes give identical results
    if strip:
        monkeypatch.setenv("BZ_TILE_S", str(strip))
    if threads:
        monkeypatch.setenv("BZ_TILE_THREADS", str(threads))
    I = gen_document(130, 1100, 8, noise=10.0, stain=True)
    check_sums(bz, I, 33, 40)
    mask, _, _ = bz.sauvola(dev(I), 33, 40, k=0.45)
    ref = oracle.sauvola(I, 33, 40, k=0.45)
    assert mask_report(mask.cpu().numpy(), ref, I) == 0
