"""The shared input generator: determinism, value ranges, ink coverage."""
import numpy as np

from docgen import gen_document, batch_specs, INK_TARGET


def test_deterministic_and_seed_dependent():
    a = gen_document(96, 128, 1)
    b = gen_document(96, 128, 1)
    c = gen_document(96, 128, 2)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_ranges_and_dtypes():
    a = gen_document(64, 80, 3, noise=10, stain=True)
    assert a.dtype == np.uint8
    f = gen_document(64, 80, 3, noise=10, stain=True, dtype=np.float32)
    assert f.dtype == np.float32 and f.min() >= 0 and f.max() <= 255
    assert np.array_equal(np.rint(f).astype(np.uint8), a)


def test_ink_coverage_and_background():
    # noise-free page: ink pixels are dark (N(50, 20)), background bright
    a = gen_document(384, 512, 1).astype(np.float64)
    dark = (a < 110).mean()
    assert abs(dark - INK_TARGET) < 0.02
    assert 150 < np.median(a) < 215
    # the illumination ramp brightens the right side
    assert a[:, -32:].mean() > a[:, :32].mean()


def test_degenerate_shapes():
    for (H, W) in [(1, 1), (1, 7), (9, 1)]:
        a = gen_document(H, W, 5)
        assert a.shape == (H, W)


def test_batch_specs():
    s = batch_specs()
    assert len(s) == 256
    assert all(256 <= d["H"] <= 4096 and 256 <= d["W"] <= 4096 for d in s)
    assert all(d["h"] == d["w"] and d["h"] % 2 == 1 and 11 <= d["h"] <= 101 for d in s)
    assert all(0.2 <= d["k"] <= 0.5 and d["R"] == 128.0 for d in s)
    assert s == batch_specs()
