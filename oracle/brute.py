"""Brute-force and exact-arithmetic forms of the oracle's definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  These are written
independently of ``oracle.c`` so that the C oracle can be pinned against them:

* ``window_offsets`` reads the window straight off the Introduction's mean
  formula, i - h/2 < a <= i + h/2 (and likewise for columns), with exact
  rational h/2;
* ``sums_shift`` adds shifted, zero-padded copies of the image, one per window
  offset (NumPy; the zero padding is Section 3.2's out-of-range convention);
* ``sums_python`` is a pure-Python loop for tiny images;
* ``exact_below_sauvola`` / ``exact_below_niblack`` decide I < t in exact
  rational arithmetic (Python integers and Fractions), with k and R taken as
  the exact values of their float32 representations.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def window_offsets(size: int):
    """Integer offsets d with -size/2 < d <= size/2 (Introduction)."""
    half = Fraction(size, 2)
    lo = int(np.floor(-half)) - 1
    return [d for d in range(lo, int(half) + 2) if -half < d <= half]


def sums_shift(I: np.ndarray, h: int, w: int):
    """S1, S2 (int64) as a sum of shifted zero-padded images."""
    I = np.asarray(I, dtype=np.int64)
    H, W = I.shape
    dr, dc = window_offsets(h), window_offsets(w)
    P = max(abs(d) for d in dr + dc) + 1
    Z = np.zeros((H + 2 * P, W + 2 * P), np.int64)
    Z[P:P + H, P:P + W] = I
    Z2 = Z * Z
    S1 = np.zeros((H, W), np.int64)
    S2 = np.zeros((H, W), np.int64)
    for a in dr:
        for b in dc:
            S1 += Z[P + a:P + a + H, P + b:P + b + W]
            S2 += Z2[P + a:P + a + H, P + b:P + b + W]
    return S1, S2


def count_shift(H: int, W: int, h: int, w: int):
    """In-bounds window element counts, by counting (sums of a ones image)."""
    return sums_shift(np.ones((H, W), np.int64), h, w)[0]


def sums_python(I, h: int, w: int):
    """Pure-Python S1, S2 and n for tiny images (lists of lists)."""
    I = [[int(v) for v in row] for row in np.asarray(I)]
    H, W = len(I), len(I[0])
    hh, ww = Fraction(h, 2), Fraction(w, 2)
    S1 = [[0] * W for _ in range(H)]
    S2 = [[0] * W for _ in range(H)]
    N = [[0] * W for _ in range(H)]
    for i in range(H):
        for j in range(W):
            for a in range(H):
                if not (i - hh < a <= i + hh):
                    continue
                for b in range(W):
                    if not (j - ww < b <= j + ww):
                        continue
                    S1[i][j] += I[a][b]
                    S2[i][j] += I[a][b] ** 2
                    N[i][j] += 1
    return np.array(S1), np.array(S2), np.array(N)


def exact_below_sauvola(I: int, S1: int, S2: int, n: int, k: float, R: float) -> bool:
    """Exact truth of I < m (1 + k (s/R - 1)) for k >= 0, R > 0, where
    m = S1/n and s^2 = (n S2 - S1^2)/n^2 (Section 3.2's squared form)."""
    k = Fraction(float(np.float32(k)))
    R = Fraction(float(np.float32(R)))
    assert k >= 0 and R > 0
    m = Fraction(S1, n)
    v = Fraction(n * S2 - S1 * S1, n * n)
    A = I - m * (1 - k)          # I - m(1 - k); condition: A < m k s / R
    if A < 0:
        return True
    rhs2 = (m * k / R) ** 2 * v  # (m k s / R)^2
    return A * A < rhs2


def exact_below_niblack(I: int, S1: int, S2: int, n: int, k: float) -> bool:
    """Exact truth of I < m + k s (any sign of k)."""
    k = Fraction(float(np.float32(k)))
    m = Fraction(S1, n)
    v = Fraction(n * S2 - S1 * S1, n * n)
    A = I - m                    # condition: A < k s
    if k >= 0:
        return A < 0 or A * A < k * k * v
    return A < 0 and A * A > k * k * v


def quantile_python(I, h: int, w: int, q: float):
    """Pure-Python windowed quantile: sort the clipped window, take the
    rho-th smallest with rho = max(1, ceil(q n)) (q n in binary64)."""
    import math
    I = np.asarray(I)
    H, W = I.shape
    dr, dc = window_offsets(h), window_offsets(w)
    Q = np.zeros((H, W), np.uint8)
    for i in range(H):
        for j in range(W):
            vals = sorted(int(I[i + a, j + b]) for a in dr for b in dc
                          if 0 <= i + a < H and 0 <= j + b < W)
            rho = max(1, math.ceil(float(q) * float(len(vals))))
            Q[i, j] = vals[rho - 1]
    return Q
