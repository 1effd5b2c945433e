"""Seeded synthetic document pages (the shared input generator).

This module is the only code that both the GPU path's tests/benchmarks and the
CPU oracle's tests use.  It draws random numbers and paints pixels; it contains
none of the binarization arithmetic (no window sums, moments, thresholds or
quantiles).

The paper measures on the DIBCO 2009/2013 contest images, which are not
available here; these pages stand in for them with document-like statistics: a
bright, unevenly lit background, thin dark strokes (about 10% ink) and,
optionally, a smooth stain field and sensor noise.

Recipe (every draw comes from ``numpy.random.default_rng(seed)``, PCG64):

1. background ~ N(200, 15^2), i.i.d. per pixel;
2. illumination ramp along the columns: background *= 0.7 + 0.3 * j / (W - 1);
3. strokes: axis-aligned rectangle outlines and straight segments at random
   angles, stroke width uniform in {1..4}, drawn until the ink coverage reaches
   10%; ink pixels take i.i.d. N(50, 20^2) values that replace the background;
4. optional stain: the sum of four Gaussian blobs with amplitudes U[-60, -20],
   centres uniform over the page and widths U[0.1, 0.3] * min(H, W);
5. additive N(0, noise^2) noise;
6. clip to [0, 255]; uint8 output is rounded to nearest (np.rint), float32
   output is not rounded.
"""
from __future__ import annotations

import numpy as np

__all__ = ["gen_document", "gen_batch", "batch_specs", "soft_batch", "INK_TARGET"]

INK_TARGET = 0.10


def _paint_strokes(ink: np.ndarray, rng: np.random.Generator, target: float) -> None:
    """Set ``ink`` (bool H x W, in place) until its mean reaches ``target``."""
    H, W = ink.shape
    total = H * W
    need = int(np.ceil(target * total))
    count = int(ink.sum())
    side = min(H, W)
    # Stroke lengths scale with the page so that one stroke never overshoots
    # the coverage target by more than a small fraction of it.
    lmax = max(4, side // 10)
    while count < need:
        width = int(rng.integers(1, 5))
        if rng.random() < 0.4:
            # rectangle outline (a glyph box / table cell)
            hh = int(rng.integers(3, lmax + 4))
            ww = int(rng.integers(3, lmax + 4))
            y0 = int(rng.integers(-hh // 2, H))
            x0 = int(rng.integers(-ww // 2, W))
            bars = (
                (y0, y0 + width, x0, x0 + ww),
                (y0 + hh - width, y0 + hh, x0, x0 + ww),
                (y0, y0 + hh, x0, x0 + width),
                (y0, y0 + hh, x0 + ww - width, x0 + ww),
            )
            ys_list, xs_list = [], []
            for a, b, c, d in bars:
                a, b = max(a, 0), min(b, H)
                c, d = max(c, 0), min(d, W)
                if a >= b or c >= d:
                    continue
                yy, xx = np.mgrid[a:b, c:d]
                ys_list.append(yy.ravel())
                xs_list.append(xx.ravel())
            if not ys_list:
                continue
            ys = np.concatenate(ys_list)
            xs = np.concatenate(xs_list)
        else:
            # straight segment of random angle (a pen stroke)
            length = float(rng.uniform(3, lmax + 3))
            theta = float(rng.uniform(0, np.pi))
            cy = float(rng.uniform(0, H))
            cx = float(rng.uniform(0, W))
            t = np.arange(-length / 2, length / 2, 0.5)
            o = np.arange(width) - (width - 1) / 2.0
            dy, dx = np.sin(theta), np.cos(theta)
            py = cy + t[:, None] * dy + o[None, :] * dx
            px = cx + t[:, None] * dx - o[None, :] * dy
            ys = np.rint(py).astype(np.int64).ravel()
            xs = np.rint(px).astype(np.int64).ravel()
            keep = (ys >= 0) & (ys < H) & (xs >= 0) & (xs < W)
            ys, xs = ys[keep], xs[keep]
            if ys.size == 0:
                continue
        flat = np.unique(ys * W + xs)
        fresh = flat[~ink.ravel()[flat]]
        if fresh.size == 0:
            continue
        ink.ravel()[fresh] = True
        count += int(fresh.size)


def gen_document(H: int, W: int, seed: int, noise: float = 0.0, stain: bool = False,
                 dtype=np.uint8) -> np.ndarray:
    """Return one synthetic page of shape (H, W) as uint8 or float32."""
    if H < 1 or W < 1:
        raise ValueError("H and W must be positive")
    rng = np.random.default_rng(seed)
    img = rng.standard_normal((H, W), dtype=np.float32)
    img *= np.float32(15.0)
    img += np.float32(200.0)
    if W > 1:
        ramp = (0.7 + 0.3 * np.arange(W, dtype=np.float64) / (W - 1)).astype(np.float32)
    else:
        ramp = np.ones(1, dtype=np.float32)
    img *= ramp[None, :]
    ink = np.zeros((H, W), dtype=bool)
    _paint_strokes(ink, rng, INK_TARGET)
    nink = int(ink.sum())
    vals = rng.standard_normal(nink, dtype=np.float32) * np.float32(20.0) + np.float32(50.0)
    img[ink] = vals
    if stain:
        side = min(H, W)
        yy = np.arange(H, dtype=np.float32)
        xx = np.arange(W, dtype=np.float32)
        for _ in range(4):
            amp = float(rng.uniform(-60.0, -20.0))
            cy = float(rng.uniform(0, H))
            cx = float(rng.uniform(0, W))
            sig = float(rng.uniform(0.1, 0.3)) * side
            gy = np.exp(-((yy - cy) ** 2) / (2 * sig * sig)).astype(np.float32)
            gx = np.exp(-((xx - cx) ** 2) / (2 * sig * sig)).astype(np.float32)
            img += np.float32(amp) * gy[:, None] * gx[None, :]
    if noise > 0:
        img += rng.standard_normal((H, W), dtype=np.float32) * np.float32(noise)
    np.clip(img, 0.0, 255.0, out=img)
    if np.dtype(dtype) == np.uint8:
        return np.rint(img).astype(np.uint8)
    if np.dtype(dtype) == np.float32:
        return img
    raise ValueError("dtype must be uint8 or float32")


def batch_specs(count: int = 256, seed: int = 4, hw_lo: int = 256, hw_hi: int = 4096,
                win_lo: int = 11, win_hi: int = 101):
    """Per-image shapes and parameters of the ragged batch workload.

    H and W uniform in [hw_lo, hw_hi]; h = w odd, uniform in [win_lo, win_hi];
    k uniform in [0.2, 0.5]; R = 128; image b uses generator seed 4000 + b.
    Returns a list of dicts.
    """
    rng = np.random.default_rng(seed)
    odd = np.arange(win_lo | 1, win_hi + 1, 2)
    specs = []
    for b in range(count):
        H = int(rng.integers(hw_lo, hw_hi + 1))
        W = int(rng.integers(hw_lo, hw_hi + 1))
        win = int(odd[rng.integers(0, odd.size)])
        k = float(np.float32(rng.uniform(0.2, 0.5)))
        specs.append(dict(H=H, W=W, h=win, w=win, k=k, R=128.0, seed=4000 + b))
    return specs


def soft_batch(B: int = 32, H: int = 1024, W: int = 1024):
    """Inputs of the differentiable workload: images, per-image k, and the
    upstream weights Wrand of the loss sum(y * Wrand).

    Images b use seeds 5000 + b (float32, noise 10, stain); k from seed 5998
    as U[0.2, 0.5]; Wrand ~ N(0, 1) from seed 5999.
    """
    imgs = np.stack([gen_document(H, W, 5000 + b, noise=10.0, stain=True, dtype=np.float32)
                     for b in range(B)])
    k = np.random.default_rng(5998).uniform(0.2, 0.5, size=B).astype(np.float32)
    wr = np.random.default_rng(5999).standard_normal((B, H, W), dtype=np.float32)
    return imgs, k, wr


def _gen_one(args):
    H, W, seed, noise, stain = args
    return gen_document(H, W, seed, noise=noise, stain=stain)


def gen_batch(specs, noise: float = 10.0, stain: bool = True, workers: int = 8):
    """uint8 pages for a list of specs (dicts with H, W, seed), generated in
    fresh worker processes (spawned interpreters) when workers > 1."""
    jobs = [(d["H"], d["W"], d["seed"], noise, stain) for d in specs]
    if workers <= 1 or len(jobs) < 4:
        return [_gen_one(j) for j in jobs]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_gen_one, jobs, chunksize=4))
