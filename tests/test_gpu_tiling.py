"""The tiling table of the single-image calls (bz_set_tile_table): outputs do
not depend on the strip heights and block sizes it picks, invalid rows are
rejected, and the tuner's cache is read back for the current device."""
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


@pytest.fixture
def clean_table(bz, monkeypatch):
    monkeypatch.delenv("BZ_TILE_S", raising=False)
    monkeypatch.delenv("BZ_TILE_THREADS", raising=False)
    bz.set_tile_table([])
    yield
    bz.set_tile_table([])


CASES = [(1000, 2500, 31), (300, 700, 75), (2048, 4096, 15), (77, 5000, 9)]


@pytest.mark.parametrize("H,W,h", CASES)
@pytest.mark.parametrize("strip,threads", [(4, 256), (13, 512), (32, 1024), (0, 64), (7, 0)])
def test_tiled_outputs_equal_the_built_in_plan(bz, clean_table, H, W, h, strip, threads):
    print("tiling", H, W, h, strip, threads, flush=True)
    img = torch.from_numpy(gen_document(H, W, H + W + h, noise=10.0, stain=True)).cuda()
    ref = [t.clone() for t in bz.sauvola(img, h, h, 0.4, 128.0)]
    S1r, S2r = bz.window_sums(img, h, h)
    # one row for the case's class, and rows for other classes that must not
    # apply to it
    bz.set_tile_table([[h - 1, 10 ** 6, 1, 64], [h, W, strip, threads], [10 ** 6, 10 ** 6, 2, 128]]
                      if h > 1 else [[h, W, strip, threads]])
    got = bz.sauvola(img, h, h, 0.4, 128.0)
    S1, S2 = bz.window_sums(img, h, h)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    assert torch.equal(S1, S1r) and torch.equal(S2, S2r)


@pytest.mark.parametrize("row", [[0, 10, 8, 256], [15, 0, 8, 256], [15, 10, -1, 256], [15, 10, 8, 100],
                                 [15, 10, 8, 2048], [15, 10, 8, -64]])
def test_invalid_rows_are_rejected(bz, clean_table, row):
    with pytest.raises(ValueError):
        bz.set_tile_table([row])


def test_cached_rows_for_this_device(bz, tmp_path):
    from paper_1905_13038_amd import tune
    p = str(tmp_path / "tilings.json")
    name = torch.cuda.get_device_name(torch.device("cuda"))
    rows = [[15, 1024, 8, 256], [257, 8192, 0, 0]]
    tune.save_table(p, name, "plain", rows)
    assert tune.cached_plain_rows(p) == rows
    with open(p, "w") as f:
        f.write("{corrupt")
    assert tune.cached_plain_rows(p) is None


def test_autotune_plain_rows_are_valid_and_installable(bz, clean_table):
    # a small measurement (two window classes, two widths, two strips, two
    # block sizes): one row per class pair, each installable, outputs
    # unchanged under the table
    from paper_1905_13038_amd import tune
    rows = tune.autotune_plain(H=256, classes=(15, 63), widths=(512, 2048), strips=(8, 24), threads=(256, 1024),
                               reps=1, cache_path=None)
    assert len(rows) == 4
    for hmax, wmax, strip, threads in rows:
        assert hmax in (15, 63) and wmax in (512, 2048)
        assert strip in (0, 8, 24) and threads in (0, 256, 1024) and (strip == 0) == (threads == 0)
    img = torch.from_numpy(gen_document(300, 1500, 77, noise=10.0, stain=True)).cuda()
    ref = [t.clone() for t in bz.sauvola(img, 41, 41)]
    bz.set_tile_table(rows)
    got = bz.sauvola(img, 41, 41)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(got, ref))
