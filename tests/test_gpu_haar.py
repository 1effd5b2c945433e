"""GPU parity of the Haar-like features (bz_haar_features) against the
oracle: exact int32 values for every template, small and ragged images, a
strided input, 1 x 1 and 257-row cells, templates as large as the image, and
the 3072 x 4096 page, for the single-launch form (at each tile width and
several strip heights) and the two-launch form."""
import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document

pytestmark = pytest.mark.gpu

KINDS = {"edge_h": oracle.HAAR_EDGE_H, "edge_v": oracle.HAAR_EDGE_V, "line_h": oracle.HAAR_LINE_H,
         "line_v": oracle.HAAR_LINE_V, "checker": oracle.HAAR_CHECKER}


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def check(bz, I, a, b, kind, view=None):
    print("haar", kind, I.shape, a, b, flush=True)
    F = bz.haar_features(torch.from_numpy(np.ascontiguousarray(I)).cuda() if view is None else view, a, b, kind)
    torch.cuda.synchronize()
    ref = oracle.haar(I, a, b, KINDS[kind])
    got = F.cpu().numpy().astype(np.int64)
    assert got.shape == ref.shape and np.array_equal(got, ref)


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("H,W,a,b", [(120, 160, 6, 8), (203, 301, 5, 9), (31, 1100, 3, 257), (600, 45, 257, 7),
                                     (17, 19, 1, 1)])
def test_haar_matches_oracle(bz, kind, H, W, a, b):
    kv, kh = bz.HAAR[kind][1]
    if kv * a > H or kh * b > W:
        pytest.skip("template larger than the image")
    check(bz, gen_document(H, W, 500 + H, noise=10.0, stain=True), a, b, kind)


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_haar_template_as_large_as_the_image(bz, kind):
    kv, kh = bz.HAAR[kind][1]
    a, b = 7, 5
    check(bz, gen_document(kv * a, kh * b, 7, noise=10.0), a, b, kind)


def test_haar_strided_input(bz):
    I = gen_document(150, 277, 11, noise=10.0, stain=True)
    big = torch.zeros((150, 290), dtype=torch.uint8, device="cuda")
    big[:, 6:283] = torch.from_numpy(I).cuda()
    for kind in sorted(KINDS):
        check(bz, I, 9, 13, kind, view=big[:, 6:283])


def test_haar_extremes_of_the_value_range(bz):
    # all-255 cells against all-0 cells at the largest size: |F| = 255 * 257^2
    a = b = 257
    I = np.zeros((257, 514), np.uint8)
    I[:, :257] = 255
    check(bz, I, a, b, "edge_h")
    check(bz, I[:, ::-1].copy(), a, b, "edge_h")
    # 257-row cells of 255 in the single-launch form (its cell sums fill 16
    # bits exactly: 255 * 257 = 65535)
    J = np.zeros((514, 300), np.uint8)
    J[:257] = 255
    check(bz, J, 257, 7, "edge_v")
    check(bz, J[::-1].copy(), 257, 7, "edge_v")
    check(bz, np.full((257 * 3, 64), 255, np.uint8), 257, 5, "line_v")


@pytest.mark.parametrize("kind,a", [("edge_h", 12), ("checker", 12), ("line_v", 12), ("line_v", 48)])
def test_haar_headline_page(bz, kind, a):
    check(bz, gen_document(3072, 4096, 2, noise=10.0, stain=True), a, a, kind)


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("ndw,strip", [(1, 1), (1, 5), (2, 3), (2, 64), (1, 1000)])
def test_haar_fused_tiles_and_strips(bz, monkeypatch, kind, ndw, strip):
    # the single-launch form at each tile width (256 or 512 columns of G per
    # wavefront) and strip height, on a page several tiles wide with a ragged
    # last tile and strip, and on an aligned strided view
    monkeypatch.setenv("BZ_HAAR_NDW", str(ndw))
    monkeypatch.setenv("BZ_HAAR_STRIP", str(strip))
    I = gen_document(211, 1337, 31, noise=10.0, stain=True)
    check(bz, I, 7, 11, kind)
    big = torch.zeros((211, 1352), dtype=torch.uint8, device="cuda")
    big[:, 8:1345] = torch.from_numpy(I).cuda()
    check(bz, I, 9, 29, kind, view=big[:, 8:1345])


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_haar_two_launch_form(bz, monkeypatch, kind):
    # BZ_HAAR_FUSED=0: the column-sum field and row kernel, on aligned rows
    monkeypatch.setenv("BZ_HAAR_FUSED", "0")
    check(bz, gen_document(203, 301, 77, noise=10.0, stain=True), 5, 9, kind)


@pytest.mark.parametrize("kind,H,W,a,b", [("edge_h", 40, 17000, 5, 257), ("line_v", 70, 6000, 20, 9),
                                          ("checker", 50, 8000, 10, 77)])
def test_haar_rows_wider_than_the_row_kernel(bz, monkeypatch, kind, H, W, a, b):
    # kv * W above 12288 (48 KiB of prefixes): the prefix and combine launches
    # of the two-launch form
    monkeypatch.setenv("BZ_HAAR_FUSED", "0")
    check(bz, gen_document(H, W, 600 + kind.__len__(), noise=10.0, stain=True), a, b, kind)


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("H,W,a,b", [(300, 400, 17, 5), (200, 256, 33, 3), (260, 132, 16, 9), (64, 64, 20, 20)])
def test_haar_fused_priming_chunks_and_tail(bz, kind, H, W, a, b):
    # cells of 16 rows or more prime in chunks of 16 rows, then the rest four
    # at a time: cell heights with and without a remainder, on aligned rows
    # (the single-launch form)
    kv, kh = bz.HAAR[kind][1]
    if kv * a > H or kh * b > W:
        pytest.skip("template larger than the image")
    check(bz, gen_document(H, W, 700 + a, noise=10.0, stain=True), a, b, kind)
