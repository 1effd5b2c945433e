"""The allocation-free Bernsen entry point (device array of the library in
place of a workspace argument) against bz_bernsen, through the C ABI: two
calls in a row, the second on a smaller image, each bit-exact."""
import numpy as np
import pytest
import torch

from docgen import gen_document

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def _bernsen_pair(bz, H, W, ld, h, w, cmin, seed):
    lib = bz.lib
    st = torch.cuda.current_stream().cuda_stream
    host = gen_document(H, ld, seed, noise=10, stain=True)
    img = torch.from_numpy(host).cuda()
    outs = {}
    for name in ("plain", "noalloc"):
        mask = torch.full((H, W), 7, dtype=torch.uint8, device="cuda")
        mn = torch.full((H, W), 7, dtype=torch.uint8, device="cuda")
        mx = torch.full((H, W), 7, dtype=torch.uint8, device="cuda")
        if name == "plain":
            nb = int(lib.bz_extremes_workspace_size(H, W))
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            rc = lib.bz_bernsen(img.data_ptr(), H, W, ld, h, w, cmin, mask.data_ptr(), W, mn.data_ptr(),
                                mx.data_ptr(), W, ws.data_ptr(), nb, st)
        else:
            rc = lib.bz_bernsen_noalloc(img.data_ptr(), H, W, ld, h, w, cmin, mask.data_ptr(), W,
                                        mn.data_ptr(), mx.data_ptr(), W, st)
        assert rc == 0, (name, rc)
        torch.cuda.synchronize()
        outs[name] = (mask.cpu().numpy(), mn.cpu().numpy(), mx.cpu().numpy())
    for a, b in zip(outs["plain"], outs["noalloc"]):
        assert np.array_equal(a, b)


def test_noalloc_equals_workspace_call_twice(bz):
    # windows above 64 take the two passes through the field, which the
    # allocation-free call keeps in the library's device array; smaller ones
    # the single-launch tile form (no field)
    print("noalloc bernsen 1536x2048 h=w=101, then 300x257 (row stride 260) h=9 w=77", flush=True)
    _bernsen_pair(bz, 1536, 2048, 2048, 101, 101, 15, 3)
    _bernsen_pair(bz, 300, 257, 260, 9, 77, 20, 4)
    print("noalloc bernsen 1536x2048 h=w=32, then 300x257 h=9 w=33", flush=True)
    _bernsen_pair(bz, 1536, 2048, 2048, 32, 32, 15, 5)
    _bernsen_pair(bz, 300, 257, 260, 9, 33, 20, 6)


def test_noalloc_rejects_images_beyond_its_array(bz):
    lib = bz.lib
    n = int(lib.bz_bernsen_noalloc_max_pixels())
    assert n == 16777216
    H, W = 4097, 4096  # one row past the limit; rejected before any device work
    p = 1 << 20  # never dereferenced: validation fails first
    rc = lib.bz_bernsen_noalloc(p, H, W, W, 3, 3, 10, p + 2 * H * W, W, p + 3 * H * W, p + 4 * H * W, W, None)
    assert rc == 4  # BZ_ERR_WORKSPACE
