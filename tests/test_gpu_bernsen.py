"""GPU parity of the window extremes and Bernsen's midrange rule against the
oracle (bit-exact: everything is integer)."""
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


# windows up to 64 x 64 take the single-launch tile form; larger ones (and
# BZ_EXT_FUSED=0) the two passes through the transposed field
CASES = [(384, 512, 31, 31, 15), (203, 301, 9, 40, 20), (1, 1, 3, 3, 0), (70, 4100, 15, 5, 30),
         (100, 90, 257, 257, 15), (64, 64, 1, 1, 0), (1536, 2048, 32, 32, 15), (130, 129, 64, 64, 10),
         (131, 200, 65, 64, 10), (200, 131, 64, 65, 10), (65, 65, 2, 63, 5), (63, 257, 64, 1, 0)]


@pytest.mark.parametrize("form", ["fused", "fused_bytes", "two_pass"])
@pytest.mark.parametrize("H,W,h,w,c", CASES)
def test_bernsen_matches_oracle(bz, monkeypatch, form, H, W, h, w, c):
    # fused: dword loads and stores where rows are 4-byte aligned (W a
    # multiple of 4 here); fused_bytes: BZ_EXT_VEC=0, byte accesses only
    monkeypatch.setenv("BZ_EXT_FUSED", "0" if form == "two_pass" else "1")
    monkeypatch.setenv("BZ_EXT_VEC", "0" if form == "fused_bytes" else "1")
    I = gen_document(H, W, 90 + H, noise=10.0, stain=True)
    print("bernsen", H, W, h, w, c, form, flush=True)
    mask, mn, mx = bz.bernsen(dev(I), h, w, c)
    torch.cuda.synchronize()
    rmask, rmn, rmx = oracle.bernsen(I, h, w, c)
    assert np.array_equal(mn.cpu().numpy(), rmn)
    assert np.array_equal(mx.cpu().numpy(), rmx)
    assert np.array_equal(mask.cpu().numpy(), rmask)


@pytest.mark.parametrize("off,ld", [(0, 2052), (4, 2056), (1, 2051), (0, 2050)])
def test_bernsen_strided_input_and_alignment(bz, off, ld):
    # aligned views take the dword tile loads, the others the byte loads
    H, W = 300, 2040
    I = gen_document(H, W, 5 + off, noise=10.0, stain=True)
    buf = torch.zeros(H * ld + off + 8, dtype=torch.uint8, device="cuda")
    view = buf[off:off + H * ld].view(H, ld)[:, :W]
    view.copy_(dev(I))
    mask, mn, mx = bz.bernsen(view, 33, 17, 12)
    torch.cuda.synchronize()
    rmask, rmn, rmx = oracle.bernsen(I, 33, 17, 12)
    assert np.array_equal(mn.cpu().numpy(), rmn) and np.array_equal(mx.cpu().numpy(), rmx)
    assert np.array_equal(mask.cpu().numpy(), rmask)


def test_minmax_strided_view(bz):
    I = gen_document(150, 211, 4, noise=10.0, stain=True)
    big = torch.zeros((150, 230), dtype=torch.uint8, device="cuda")
    big[:, 7:218] = dev(I)
    mn, mx = bz.window_minmax(big[:, 7:218], 11, 6)
    torch.cuda.synchronize()
    _, rmn, rmx = oracle.bernsen(I, 11, 6, 0)
    assert np.array_equal(mn.cpu().numpy(), rmn) and np.array_equal(mx.cpu().numpy(), rmx)
