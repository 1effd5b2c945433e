"""Pins of the oracle's Haar-like features: SciPy's 2-D correlation with the
+-1 template, brute force over slices on tiny images, the impulse response,
constant images and the mirror antisymmetry of the two-cell features."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle
from docgen import gen_document

KINDS = sorted(oracle.HAAR_SIGNS)


def template(kind, a, b):
    return np.kron(np.array(oracle.HAAR_SIGNS[kind], np.int64), np.ones((a, b), np.int64))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("H,W,a,b", [(40, 57, 3, 4), (31, 29, 5, 2), (12, 80, 1, 1), (64, 64, 10, 7)])
def test_haar_equals_correlation_with_template(kind, H, W, a, b):
    I = gen_document(H, W, 300 + H + W, noise=10.0, stain=True)
    F = oracle.haar(I, a, b, kind)
    ref = correlate2d(I.astype(np.int64), template(kind, a, b), mode="valid")
    assert F.shape == ref.shape and np.array_equal(F, ref)


@pytest.mark.parametrize("kind", KINDS)
def test_haar_brute_force_tiny(kind):
    rng = np.random.default_rng(kind)
    for (H, W, a, b) in [(6, 7, 1, 2), (7, 9, 2, 1), (9, 9, 3, 3), (6, 6, 2, 2)]:
        I = rng.integers(0, 256, size=(H, W))
        signs = oracle.HAAR_SIGNS[kind]
        kv, kh = len(signs), len(signs[0])
        if kv * a > H or kh * b > W:
            continue
        F = oracle.haar(I.astype(np.uint8), a, b, kind)
        for i in range(H - kv * a + 1):
            for j in range(W - kh * b + 1):
                want = 0
                for m in range(kv):
                    for n in range(kh):
                        want += signs[m][n] * int(I[i + m * a:i + (m + 1) * a, j + n * b:j + (n + 1) * b].sum())
                assert F[i, j] == want


@pytest.mark.parametrize("kind", KINDS)
def test_haar_impulse_response(kind):
    # a single 1 at (p, q): F[i, j] is the sign of the cell holding (p - i, q - j)
    a, b, H, W, p, q = 3, 2, 20, 22, 9, 11
    I = np.zeros((H, W), np.uint8)
    I[p, q] = 1
    F = oracle.haar(I, a, b, kind)
    T = template(kind, a, b)
    for i in range(F.shape[0]):
        for j in range(F.shape[1]):
            di, dj = p - i, q - j
            inside = 0 <= di < T.shape[0] and 0 <= dj < T.shape[1]
            assert F[i, j] == (T[di, dj] if inside else 0)


def test_haar_constant_image():
    c, a, b = 77, 4, 5
    I = np.full((30, 40), c, np.uint8)
    for kind in (oracle.HAAR_EDGE_H, oracle.HAAR_EDGE_V, oracle.HAAR_CHECKER):
        assert not oracle.haar(I, a, b, kind).any()
    for kind in (oracle.HAAR_LINE_H, oracle.HAAR_LINE_V):
        assert np.all(oracle.haar(I, a, b, kind) == c * a * b)


def test_haar_mirror_antisymmetry():
    I = gen_document(33, 47, 9, noise=10.0)
    Fh = oracle.haar(I, 4, 5, oracle.HAAR_EDGE_H)
    assert np.array_equal(oracle.haar(I[:, ::-1], 4, 5, oracle.HAAR_EDGE_H), -Fh[:, ::-1])
    Fv = oracle.haar(I, 4, 5, oracle.HAAR_EDGE_V)
    assert np.array_equal(oracle.haar(I[::-1, :], 4, 5, oracle.HAAR_EDGE_V), -Fv[::-1, :])


def test_haar_template_must_fit():
    with pytest.raises(ValueError):
        oracle.haar(np.zeros((5, 5), np.uint8), 3, 3, oracle.HAAR_EDGE_H)
