"""GPU parity of the windowed quantiles and their masks (bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(bz, I, h, w, q):
    Q, mask = bz.window_quantile(dev(I), h, w, q)
    return Q.cpu().numpy(), mask.cpu().numpy()


# odd widths give rows at every byte alignment; w = 189 and 201 take two
# dwords of row bytes per lane, 257 x 257 windows one 32-bit word per bin;
# windows wider than 32 build their first window four rows per pass, and the
# last three cases leave 0, 1, 2 or 3 rows over in the strips' builds
@pytest.mark.parametrize("H,W,h,w,q", [(37, 61, 8, 12, 0.1), (64, 64, 32, 32, 0.5), (50, 130, 101, 101, 0.1),
                                       (25, 70, 1, 1, 0.5), (45, 45, 16, 5, 0.75), (9, 200, 3, 40, 1.0),
                                       (200, 9, 40, 3, 0.0), (1, 1, 5, 5, 0.5), (30, 397, 9, 189, 0.5),
                                       (41, 333, 5, 201, 0.25), (270, 301, 257, 257, 0.5),
                                       (60, 150, 8, 36, 0.5), (70, 90, 12, 33, 0.3), (77, 140, 7, 35, 0.9)])
def test_small_shapes(bz, H, W, h, w, q):
    I = gen_document(H, W, H * 31 + W, noise=10, stain=True)
    Q, mask = run(bz, I, h, w, q)
    rq, rm = oracle.quantile_hist(I, h, w, q)
    assert np.array_equal(Q, rq) and np.array_equal(mask, rm)


@pytest.mark.parametrize("win", [32, 101])
@pytest.mark.parametrize("q", [0.5, 0.1])
def test_full_size(bz, win, q):
    # the 2048 x 1536 page of the quantile workload
    print("quantile full size", win, q, flush=True)
    I = gen_document(1536, 2048, 3, noise=10.0, stain=True)
    Q, mask = run(bz, I, win, win, q)
    rq, rm = oracle.quantile_hist(I, win, win, q)
    assert np.array_equal(Q, rq), int((Q != rq).sum())
    assert np.array_equal(mask, rm)


def test_constant_and_extremes(bz):
    I = np.full((40, 300), 77, np.uint8)
    Q, mask = run(bz, I, 9, 9, 0.3)
    assert np.all(Q == 77) and not mask.any()
    J = np.random.default_rng(0).integers(0, 256, size=(120, 130), dtype=np.uint8)
    for q in (0.0, 1.0, 0.5):
        Q, mask = run(bz, J, 7, 6, q)
        rq, rm = oracle.quantile_sort(J, 7, 6, q)
        assert np.array_equal(Q, rq) and np.array_equal(mask, rm)


@pytest.mark.parametrize("off,ld", [(1, 203), (3, 256), (2, 201)])
def test_unaligned_strided(bz, off, ld):
    # base offsets and row strides that put the row spans at every byte
    # alignment (the row bytes are read as aligned dwords)
    H, W = 90, 200
    buf = np.random.default_rng(off * 1000 + ld).integers(0, 256, size=(H * ld + off + 8,), dtype=np.uint8)
    d = dev(buf)
    view = d[off:off + H * ld].view(H, ld)[:, :W]
    host = np.ascontiguousarray(buf[off:off + H * ld].reshape(H, ld)[:, :W])
    Q, mask = bz.window_quantile(view, 15, 21, 0.3)
    rq, rm = oracle.quantile_hist(host, 15, 21, 0.3)
    assert np.array_equal(Q.cpu().numpy(), rq) and np.array_equal(mask.cpu().numpy(), rm)
