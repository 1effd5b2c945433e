"""CPU oracle for local adaptive binarization statistics.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library under ``paper_1905_13038_amd``.

``oracle.c`` (plain C, binary64, built with ``-ffp-contract=off``) holds the
definitions; this module loads it with ctypes and adds NumPy conveniences.
``brute.py`` holds pure-Python forms for tiny inputs and exact rational
decisions.  Function docstrings cite the paper passage each one follows.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
(brute force, integral images, closed forms, invariants, library order
statistics and correlations, finite differences); none is "parity unpinned" except the choice
of quantile definition itself (the paper does not define one; the inverse
empirical CDF is used).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MEANSTD, SAUVOLA, NIBLACK = 0, 1, 2
# the remaining methods of Table 1
WOLF, FENG, RAIS, NICK, PHANSALKAR = 3, 4, 5, 6, 7
TABLE1_PARAMS = {WOLF: ("k", "R"), FENG: ("a1", "k1", "k2", "gamma", "R"), RAIS: (),
                 NICK: ("k",), PHANSALKAR: ("p", "q", "k", "R")}

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (no fast-math, no
    contraction: every binary64 operation rounds once)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """Compile ``oracle.c`` with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only) into ``out``, for running the pins under the sanitizers
    (the process must preload the ASan runtime; ``ORACLE_LIB=out`` makes this
    module load it)."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wall", "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB")
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, f32, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    lib.orc_count.restype = i64
    lib.orc_count.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.orc_sums_direct.restype = None
    lib.orc_sums_direct.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.orc_sums_direct_at.restype = None
    lib.orc_sums_direct_at.argtypes = [P, i32, i32, i64, i32, i32, i32, P, P, P, P]
    lib.orc_sums_recursive.restype = i32
    lib.orc_sums_recursive.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.orc_sums_integral.restype = i32
    lib.orc_sums_integral.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.orc_threshold.restype = None
    lib.orc_threshold.argtypes = [P, i32, i32, i64, i32, i32, P, P, i32, f32, f32, P, P, P, P]
    lib.orc_global_stats.restype = None
    lib.orc_global_stats.argtypes = [P, i32, i32, i64, P, P]
    lib.orc_table1_t.restype = f64
    lib.orc_table1_t.argtypes = [i32, f64, f64, f64, P, f64, f64, f64]
    lib.orc_table1.restype = None
    lib.orc_table1.argtypes = [P, i32, i32, i64, i32, i32, P, P, i32, P, P, P, P]
    lib.orc_sauvola_sqrtfree.restype = None
    lib.orc_sauvola_sqrtfree.argtypes = [P, i32, i32, i64, i32, i32, P, P, f32, f32, P]
    lib.orc_rank.restype = i64
    lib.orc_rank.argtypes = [f64, i64]
    lib.orc_quantile_sort.restype = None
    lib.orc_quantile_sort.argtypes = [P, i32, i32, i64, i32, i32, f64, P, P]
    lib.orc_quantile_hist.restype = None
    lib.orc_quantile_hist.argtypes = [P, i32, i32, i64, i32, i32, f64, P, P]
    lib.orc_soft_fwd.restype = None
    lib.orc_soft_fwd.argtypes = [P, i32, i32, i32, i32, i32, P, f64, f64, P, P]
    lib.orc_box_f64.restype = None
    lib.orc_box_f64.argtypes = [P, i32, i32, i32, i32, P]
    lib.orc_box_adjoint.restype = None
    lib.orc_box_adjoint.argtypes = [P, i32, i32, i32, i32, P]
    lib.orc_soft_bwd.restype = None
    lib.orc_soft_bwd.argtypes = [P, P, i32, i32, i32, i32, i32, P, f64, f64, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _img(I: np.ndarray):
    """Return (array, H, W, ld) for a 2-D uint8 view with unit column stride."""
    I = np.asarray(I)
    if I.dtype != np.uint8 or I.ndim != 2:
        raise TypeError("expected a 2-D uint8 image")
    if I.strides[1] != 1:
        I = np.ascontiguousarray(I)
    H, W = I.shape
    ld = I.strides[0] if H > 1 else W
    return I, H, W, ld


def extents(h: int, w: int):
    """(o, u, l, r) of Algorithm 1."""
    return (h + 1) // 2, h // 2, (w + 1) // 2, w // 2


def count(H: int, W: int, h: int, w: int, i: int, j: int) -> int:
    """In-bounds window count n of Algorithm 1."""
    return int(_load().orc_count(H, W, h, w, i, j))


def count_map(H: int, W: int, h: int, w: int) -> np.ndarray:
    """n for every pixel (int64, H x W): the product of Algorithm 1's row and
    column factors."""
    o, u, l, r = extents(h, w)
    i = np.arange(H)
    j = np.arange(W)
    nr = np.minimum(i + u, H - 1) - np.maximum(i - o, -1)
    nc = np.minimum(j + r, W - 1) - np.maximum(j - l, -1)
    return nr[:, None].astype(np.int64) * nc[None, :].astype(np.int64)


def sums_direct(I, h: int, w: int):
    """S1, S2 (uint64) by the direct definition of the Introduction."""
    I, H, W, ld = _img(I)
    S1 = np.empty((H, W), np.uint64)
    S2 = np.empty((H, W), np.uint64)
    _load().orc_sums_direct(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2))
    return S1, S2


def sums_direct_at(I, h: int, w: int, ii, jj):
    """S1, S2 at the listed pixels only (direct definition)."""
    I, H, W, ld = _img(I)
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    S1 = np.empty(ii.size, np.uint64)
    S2 = np.empty(ii.size, np.uint64)
    _load().orc_sums_direct_at(_ptr(I), H, W, ld, h, w, ii.size, _ptr(ii), _ptr(jj),
                               _ptr(S1), _ptr(S2))
    return S1, S2


def sums_recursive(I, h: int, w: int):
    """S1, S2 (uint32) by Algorithm 1's recursive sweep (16/32-bit
    accumulators of Section 3.3)."""
    I, H, W, ld = _img(I)
    S1 = np.empty((H, W), np.uint32)
    S2 = np.empty((H, W), np.uint32)
    rc = _load().orc_sums_recursive(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2))
    if rc != 0:
        raise ValueError("recursive sums need h, w <= 257")
    return S1, S2


def sums_integral(I, h: int, w: int):
    """S1, S2 (uint64) from two 64-bit integral images (Section 2)."""
    I, H, W, ld = _img(I)
    S1 = np.empty((H, W), np.uint64)
    S2 = np.empty((H, W), np.uint64)
    rc = _load().orc_sums_integral(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2))
    if rc != 0:
        raise MemoryError("integral image allocation failed")
    return S1, S2


def threshold(I, h: int, w: int, method: int, k: float = 0.0, R: float = 128.0,
              S1=None, S2=None):
    """Canonical binary64 moments, threshold and mask (mask = 1 iff I < t).

    Returns dict(m, s, t, mask, S1, S2).  ``k`` and ``R`` are rounded to
    float32 first, as the C-ABI takes them."""
    I, H, W, ld = _img(I)
    if S1 is None:
        S1, S2 = sums_recursive(I, h, w) if max(h, w) <= 257 else sums_integral(I, h, w)
    S1 = np.ascontiguousarray(S1, dtype=np.uint64)
    S2 = np.ascontiguousarray(S2, dtype=np.uint64)
    m = np.empty((H, W), np.float64)
    s = np.empty((H, W), np.float64)
    t = np.empty((H, W), np.float64)
    mask = np.empty((H, W), np.uint8)
    _load().orc_threshold(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2), method,
                          float(np.float32(k)), float(np.float32(R)),
                          _ptr(m), _ptr(s), _ptr(t), _ptr(mask))
    return dict(m=m, s=s, t=t, mask=mask, S1=S1, S2=S2)


def sauvola(I, h, w, k=0.5, R=128.0, **kw):
    """Sauvola (Introduction; Table 1) in the canonical binary64 sequence."""
    return threshold(I, h, w, SAUVOLA, k, R, **kw)


def niblack(I, h, w, k=-0.2, **kw):
    """Niblack (Table 1) in the canonical binary64 sequence."""
    return threshold(I, h, w, NIBLACK, k, 128.0, **kw)


def bernsen(I, h: int, w: int, contrast_min: int):
    """Bernsen's rule on the window extremes (the paper cites it as the
    midrange method computed from local minima and maxima): mn, mx = the
    clipped window's minimum and maximum (the quantiles q = 0 and q = 1);
    mask = 1 where mx - mn >= contrast_min and I lies below the midrange,
    2 I < mn + mx (exact in integers); windows of lower contrast are
    background (mask 0).  Returns (mask, mn, mx)."""
    mn, _ = quantile_hist(I, h, w, 0.0)
    mx, _ = quantile_hist(I, h, w, 1.0)
    Ii = np.asarray(I).astype(np.int32)
    lo, hi = mn.astype(np.int32), mx.astype(np.int32)
    mask = ((hi - lo >= int(contrast_min)) & (2 * Ii < lo + hi)).astype(np.uint8)
    return mask, mn, mx


# Haar-like features (the rectangle features of Viola and Jones, which the
# paper names as a use of recursive window sums): the sign of each a x b cell
# of the template, row by row
HAAR_EDGE_H, HAAR_EDGE_V, HAAR_LINE_H, HAAR_LINE_V, HAAR_CHECKER = 1, 2, 3, 4, 5
HAAR_SIGNS = {HAAR_EDGE_H: ((1, -1),), HAAR_EDGE_V: ((1,), (-1,)), HAAR_LINE_H: ((1, -1, 1),),
              HAAR_LINE_V: ((1,), (-1,), (1,)), HAAR_CHECKER: ((1, -1), (-1, 1))}


def haar(I, a: int, b: int, kind: int):
    """Haar-like feature of one template at every anchor where it fits in the
    image (Section 3.4 names these features as computable from window sums
    without integral images): the template is a grid of a x b cells with
    signs HAAR_SIGNS[kind]; F[i, j] = sum over cells (m, n) of sign(m, n)
    times the sum of I over rows i + m a .. i + (m+1) a - 1 and columns
    j + n b .. j + (n+1) b - 1.  F has H - kv a + 1 rows and W - kh b + 1
    columns (kv x kh cells).  Each cell sum is taken from the int64 integral
    image of Section 2 (Z[i, j] = sum of I over rows < i and columns < j; a
    rectangle's sum is a signed sum of its four corners)."""
    X = np.asarray(I).astype(np.int64)
    H, W = X.shape
    signs = HAAR_SIGNS[kind]
    kv, kh = len(signs), len(signs[0])
    Hf, Wf = H - kv * a + 1, W - kh * b + 1
    if Hf < 1 or Wf < 1:
        raise ValueError("the template does not fit in the image")
    Z = np.zeros((H + 1, W + 1), np.int64)
    Z[1:, 1:] = X.cumsum(0).cumsum(1)
    F = np.zeros((Hf, Wf), np.int64)
    for m in range(kv):
        for n in range(kh):
            r, c = m * a, n * b
            cell = (Z[r + a:r + a + Hf, c + b:c + b + Wf] - Z[r:r + Hf, c + b:c + b + Wf]
                    - Z[r + a:r + a + Hf, c:c + Wf] + Z[r:r + Hf, c:c + Wf])
            F += signs[m][n] * cell
    return F


def global_stats(I):
    """Table 1's global statistics of the whole image: dict(L, max, M, S, N,
    T1, T2) with L the minimum gray level, M the mean and S the population
    standard deviation (exact integer sums, then one binary64 sequence)."""
    I, H, W, ld = _img(I)
    out = np.empty(4, np.float64)
    sums = np.empty(3, np.uint64)
    _load().orc_global_stats(_ptr(I), H, W, ld, _ptr(out), _ptr(sums))
    return dict(L=out[0], max=out[1], M=out[2], S=out[3], N=int(sums[0]), T1=int(sums[1]),
                T2=int(sums[2]))


def table1_params(method: int, params):
    """The method's parameter vector (binary64) from a dict or a sequence."""
    names = TABLE1_PARAMS[method]
    if isinstance(params, dict):
        vals = [float(params[n]) for n in names]
    else:
        vals = [float(v) for v in params]
        if len(vals) != len(names):
            raise ValueError("method %d takes %d parameters" % (method, len(names)))
    return np.array(vals + [0.0] * (5 - len(vals)), np.float64)


def table1_t(method: int, m: float, s: float, n: float, params, L=0.0, M=0.0, S=0.0) -> float:
    """One threshold of Table 1 from m, s, the count n and the global L, M, S."""
    p = table1_params(method, params)
    return float(_load().orc_table1_t(method, m, s, n, _ptr(p), L, M, S))


def table1(I, h: int, w: int, method: int, params, gstats=None, S1=None, S2=None):
    """Wolf, Feng, Rais, Khurshid (NICK) or Phansalkar (Table 1): the canonical
    binary64 moments, the method's threshold and mask = 1 iff I < t.
    Returns dict(t, mask, m, s, gstats)."""
    I, H, W, ld = _img(I)
    if S1 is None:
        S1, S2 = sums_recursive(I, h, w) if max(h, w) <= 257 else sums_integral(I, h, w)
    S1 = np.ascontiguousarray(S1, dtype=np.uint64)
    S2 = np.ascontiguousarray(S2, dtype=np.uint64)
    if gstats is None:
        gstats = global_stats(I)
    g = np.array([gstats["L"], gstats["max"], gstats["M"], gstats["S"]], np.float64)
    p = table1_params(method, params)
    t = np.empty((H, W), np.float64)
    mask = np.empty((H, W), np.uint8)
    _load().orc_table1(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2), method, _ptr(p), _ptr(g),
                       _ptr(t), _ptr(mask))
    base = threshold(I, h, w, MEANSTD, S1=S1, S2=S2)
    return dict(t=t, mask=mask, m=base["m"], s=base["s"], gstats=gstats, S1=S1, S2=S2)


def sauvola_sqrtfree(I, h: int, w: int, k: float, R: float, S1=None, S2=None):
    """Section 3.2's square-root-free decision; returns the paper's output bit
    (1 = background, i.e. I > t away from ties)."""
    I, H, W, ld = _img(I)
    if S1 is None:
        S1, S2 = sums_integral(I, h, w)
    S1 = np.ascontiguousarray(S1, dtype=np.uint64)
    S2 = np.ascontiguousarray(S2, dtype=np.uint64)
    out = np.empty((H, W), np.uint8)
    _load().orc_sauvola_sqrtfree(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2),
                                 float(np.float32(k)), float(np.float32(R)), _ptr(out))
    return out


def rank(q: float, n: int) -> int:
    """rho = max(1, ceil(q * n)) with q * n in binary64."""
    return int(_load().orc_rank(float(q), int(n)))


def quantile_sort(I, h: int, w: int, q: float):
    """Windowed quantile by sorting each clipped window (the definition)."""
    I, H, W, ld = _img(I)
    Q = np.empty((H, W), np.uint8)
    mask = np.empty((H, W), np.uint8)
    _load().orc_quantile_sort(_ptr(I), H, W, ld, h, w, float(q), _ptr(Q), _ptr(mask))
    return Q, mask


def quantile_hist(I, h: int, w: int, q: float):
    """Windowed quantile by sliding 256-bin histograms (Section 3.4)."""
    I, H, W, ld = _img(I)
    Q = np.empty((H, W), np.uint8)
    mask = np.empty((H, W), np.uint8)
    _load().orc_quantile_hist(_ptr(I), H, W, ld, h, w, float(q), _ptr(Q), _ptr(mask))
    return Q, mask


def box_f64(x, h: int, w: int):
    """Window sum B x of a binary64 field over each clipped window (direct)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    H, W = x.shape
    out = np.empty((H, W), np.float64)
    _load().orc_box_f64(_ptr(x), H, W, h, w, _ptr(out))
    return out


def box_adjoint(G, h: int, w: int):
    """Adjoint B* G of the window sum: the sum of G over the centres whose
    window contains each pixel (the reflected, clipped window)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    H, W = G.shape
    out = np.empty((H, W), np.float64)
    _load().orc_box_adjoint(_ptr(G), H, W, h, w, _ptr(out))
    return out


def soft_fwd(I, h: int, w: int, k, R: float, tau: float):
    """Soft Sauvola forward in binary64: y = sigmoid((I - t) / tau) for a
    (B, H, W) float32 stack; returns (y, t)."""
    I = np.ascontiguousarray(I, dtype=np.float32)
    if I.ndim == 2:
        I = I[None]
    B, H, W = I.shape
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.float64), (B,)))
    y = np.empty((B, H, W), np.float64)
    t = np.empty((B, H, W), np.float64)
    _load().orc_soft_fwd(_ptr(I), B, H, W, h, w, _ptr(k), float(R), float(tau), _ptr(y), _ptr(t))
    return y, t


def soft_bwd(I, g, h: int, w: int, k, R: float, tau: float):
    """Gradients of sum(g * y) w.r.t. I, k (per image) and R, binary64."""
    I = np.ascontiguousarray(I, dtype=np.float32)
    if I.ndim == 2:
        I = I[None]
    B, H, W = I.shape
    g = np.ascontiguousarray(np.broadcast_to(np.asarray(g, np.float64), (B, H, W)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.float64), (B,)))
    gI = np.empty((B, H, W), np.float64)
    gk = np.empty(B, np.float64)
    gR = np.empty(1, np.float64)
    _load().orc_soft_bwd(_ptr(I), _ptr(g), B, H, W, h, w, _ptr(k), float(R), float(tau),
                         _ptr(gI), _ptr(gk), _ptr(gR))
    return gI, gk, float(gR[0])


def time_recursive_sauvola(I, h: int, w: int, k: float, R: float, min_seconds: float = 10.0):
    """Wall-clock Mpix/s of the oracle's Algorithm 1 sweep plus the canonical
    threshold on one thread (repeated until ``min_seconds`` have passed).
    Returns (mpix_per_s, repeats, seconds)."""
    I, H, W, ld = _img(I)
    lib = _load()
    S1 = np.empty((H, W), np.uint32)
    S2 = np.empty((H, W), np.uint32)
    S1w = np.empty((H, W), np.uint64)
    S2w = np.empty((H, W), np.uint64)
    m = np.empty((H, W), np.float64)
    s = np.empty((H, W), np.float64)
    mask = np.empty((H, W), np.uint8)
    reps = 0
    t0 = time.perf_counter()
    while True:
        lib.orc_sums_recursive(_ptr(I), H, W, ld, h, w, _ptr(S1), _ptr(S2))
        np.copyto(S1w, S1)
        np.copyto(S2w, S2)
        lib.orc_threshold(_ptr(I), H, W, ld, h, w, _ptr(S1w), _ptr(S2w), SAUVOLA,
                          float(np.float32(k)), float(np.float32(R)), _ptr(m), _ptr(s),
                          None, _ptr(mask))
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return reps * H * W / dt / 1e6, reps, dt



def _bands(I, h: int, w: int, threads: int):
    """Row bands for a threaded run: output rows y0..y1-1 of each band, and
    its input rows a..e-1 (the window's halo, o - 1 rows above and u below,
    clipped to the image), copied as an image of their own."""
    I, H, W, ld = _img(I)
    o, u, _, _ = extents(h, w)
    edges = [H * t // threads for t in range(threads + 1)]
    out = []
    for t in range(threads):
        y0, y1 = edges[t], edges[t + 1]
        if y1 > y0:
            a, e = max(y0 - o + 1, 0), min(y1 + u, H)
            out.append((y0, y1, a, np.ascontiguousarray(I[a:e])))
    return out


class _BandRun:
    """The oracle's Algorithm 1 sweep and canonical Sauvola threshold on one
    band, with buffers reused across runs."""

    def __init__(self, sub, h, w, k, R):
        self.sub, self.h, self.w = sub, h, w
        self.k, self.R = float(np.float32(k)), float(np.float32(R))
        Hb, W = sub.shape
        self.S1 = np.empty((Hb, W), np.uint32)
        self.S2 = np.empty((Hb, W), np.uint32)
        self.S1w = np.empty((Hb, W), np.uint64)
        self.S2w = np.empty((Hb, W), np.uint64)
        self.m = np.empty((Hb, W), np.float64)
        self.s = np.empty((Hb, W), np.float64)
        self.mask = np.empty((Hb, W), np.uint8)

    def __call__(self):
        lib = _load()
        Hb, W = self.sub.shape
        lib.orc_sums_recursive(_ptr(self.sub), Hb, W, W, self.h, self.w, _ptr(self.S1), _ptr(self.S2))
        np.copyto(self.S1w, self.S1)
        np.copyto(self.S2w, self.S2)
        lib.orc_threshold(_ptr(self.sub), Hb, W, W, self.h, self.w, _ptr(self.S1w), _ptr(self.S2w),
                          SAUVOLA, self.k, self.R, _ptr(self.m), _ptr(self.s), None, _ptr(self.mask))


def sauvola_bands(I, h: int, w: int, k: float, R: float, threads: int):
    """The Sauvola mask computed band by band on a thread pool (each band an
    image of its own with its halo rows): equal to ``sauvola(I, ...)["mask"]``,
    since every output row's window lies inside its band's input rows or is
    clipped at the same image border."""
    from concurrent.futures import ThreadPoolExecutor
    I = np.ascontiguousarray(I, dtype=np.uint8)
    bands = _bands(I, h, w, threads)
    runs = [_BandRun(sub, h, w, k, R) for (_, _, _, sub) in bands]
    with ThreadPoolExecutor(max_workers=len(runs)) as ex:
        list(ex.map(lambda r: r(), runs))
    mask = np.empty(I.shape, np.uint8)
    for (y0, y1, a, _), r in zip(bands, runs):
        mask[y0:y1] = r.mask[y0 - a:y1 - a]
    return mask


def time_recursive_sauvola_bands(I, h: int, w: int, k: float, R: float, threads: int,
                                 min_seconds: float = 10.0):
    """Wall-clock Mpix/s of ``sauvola_bands``' work (the oracle calls of
    ``time_recursive_sauvola`` on ``threads`` row bands at once; the C calls
    release the interpreter lock).  Returns (mpix_per_s, repeats, seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    I = np.ascontiguousarray(I, dtype=np.uint8)
    H, W = I.shape
    runs = [_BandRun(sub, h, w, k, R) for (_, _, _, sub) in _bands(I, h, w, threads)]
    reps = 0
    with ThreadPoolExecutor(max_workers=len(runs)) as ex:
        t0 = time.perf_counter()
        while True:
            list(ex.map(lambda r: r(), runs))
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                break
    return reps * H * W / dt / 1e6, reps, dt
