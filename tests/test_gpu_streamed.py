"""GPU parity of the banded host-memory path (bz_binarize_streamed) against
the oracle: the image streams through the device in bands of rows or
columns, each with the window's halo, and the mask must equal the
whole-image oracle's bit for bit, for row and column bands, bands narrower
than the window, one-line bands, a single band, strided host buffers and
in-place binarization of page-locked memory."""
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


def ref_mask(I, h, w, method, k, R):
    if method == "sauvola":
        return oracle.sauvola(I, h, w, k=k, R=R)["mask"]
    return oracle.niblack(I, h, w, k=k)["mask"]


def run(bz, I, h, w, method, k, R=128.0, band=None, axis="auto", pinned=False):
    print("streamed", method, I.shape, h, w, "band", band, axis, "pinned", pinned, flush=True)
    src = torch.from_numpy(np.ascontiguousarray(I))
    if pinned:
        src = src.pin_memory()
    got = bz.binarize_streamed(src, h, w, method, k, R, band=band, axis=axis).numpy()
    ref = ref_mask(I, h, w, method, k, R)
    bad = int((got != ref).sum())
    assert bad == 0, ("mask disagreements", bad)


@pytest.mark.parametrize("H,W,h,w,method,k,band,axis", [
    (700, 300, 31, 31, "sauvola", 0.5, 64, "auto"),      # row bands, ragged last band
    (250, 900, 15, 41, "niblack", -0.2, 100, "columns"),  # column bands
    (250, 900, 15, 41, "niblack", -0.2, 100, "auto"),     # a wide image in row bands
    (400, 120, 75, 75, "sauvola", 0.3, 7, "rows"),        # bands far narrower than the window
    (120, 400, 75, 75, "sauvola", 0.3, 7, "columns"),
    (60, 40, 9, 5, "niblack", 0.1, 1, "rows"),            # one line per band
    (40, 60, 5, 9, "niblack", 0.1, 1, "columns"),
    (130, 90, 32, 32, "sauvola", 0.5, 50, "rows"),        # even window: asymmetric halo
    (90, 130, 32, 18, "sauvola", 0.5, 33, "columns"),     # even window across column bands
    (100, 80, 1, 1, "sauvola", 0.5, 13, "auto"),          # 1 x 1 windows: no halo
    (300, 200, 25, 25, "sauvola", 0.5, 1000, "auto"),     # a single band
    (1, 500, 5, 7, "niblack", -0.2, 64, "columns"),       # one row, column bands
    (500, 1, 7, 5, "niblack", -0.2, 64, "rows"),          # one column, row bands
])
def test_streamed_matches_oracle(bz, H, W, h, w, method, k, band, axis):
    I = gen_document(H, W, 90 + H + W, noise=10.0, stain=True)
    run(bz, I, h, w, method, k, band=band, axis=axis)


def test_streamed_in_place_pinned(bz):
    # the mask overwrites the image it is computed from
    for (H, W, h, w, band, axis) in [(500, 260, 41, 41, 37, "rows"), (180, 640, 21, 55, 45, "columns"),
                                     (180, 640, 21, 55, 45, "rows")]:
        I = gen_document(H, W, 7 + H, noise=10.0, stain=True)
        print("in place", I.shape, h, w, "band", band, axis, flush=True)
        buf = torch.from_numpy(I.copy()).pin_memory()
        out = bz.binarize_streamed(buf, h, w, "sauvola", 0.4, 128.0, out=buf, band=band, axis=axis)
        assert out.data_ptr() == buf.data_ptr()
        assert np.array_equal(buf.numpy(), ref_mask(I, h, w, "sauvola", 0.4, 128.0))


def test_streamed_strided_host_buffers(bz):
    # image and mask at their own row strides; the padding stays untouched
    for (H, W, h, w, band, axis) in [(333, 211, 17, 23, 40, "rows"), (150, 401, 27, 11, 64, "columns")]:
        I = gen_document(H, W, 3 + W, noise=10.0, stain=True)
        big = torch.full((H, W + 13), 7, dtype=torch.uint8)
        big[:, 5:5 + W] = torch.from_numpy(I)
        outbig = torch.full((H, W + 29), 201, dtype=torch.uint8)
        print("strided", I.shape, h, w, "band", band, axis, flush=True)
        bz.binarize_streamed(big[:, 5:5 + W], h, w, "niblack", -0.25, out=outbig[:, 3:3 + W], band=band, axis=axis)
        assert np.array_equal(outbig[:, 3:3 + W].numpy(), ref_mask(I, h, w, "niblack", -0.25, 128.0))
        assert bool((outbig[:, :3] == 201).all()) and bool((outbig[:, 3 + W:] == 201).all())
        assert bool((big[:, :5] == 7).all()) and np.array_equal(big[:, 5:5 + W].numpy(), I)


def test_streamed_headline_page_equals_device_call(bz):
    # 3072 x 4096 at w = 75, pinned, in row and in column bands: equal to the
    # device call on the resident image and to the oracle
    I = gen_document(3072, 4096, 2, noise=10.0, stain=True)
    src = torch.from_numpy(I).pin_memory()
    print("headline streamed", flush=True)
    dmask, _, _ = bz.sauvola(src.cuda(), 75, 75, k=0.5, R=128.0)
    torch.cuda.synchronize()
    dmask = dmask.cpu()
    assert np.array_equal(dmask.numpy(), ref_mask(I, 75, 75, "sauvola", 0.5, 128.0))
    for band, axis in [(384, "rows"), (512, "columns"), (None, "auto")]:
        print("  band", band, axis, flush=True)
        got = bz.binarize_streamed(src, 75, 75, "sauvola", 0.5, 128.0, band=band, axis=axis)
        assert torch.equal(got, dmask)
