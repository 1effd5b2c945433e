"""Strip-height autotuner for ragged batches.

A batched launch processes each image in tiles of one strip of rows; every
strip first primes its column sums over the h - 1 rows above and below its
first row, so short strips waste priming work and tall strips leave fewer
tiles to balance across the persistent grid.  ``autotune`` measures, per
window-size class, the batch time of a few candidate strip heights on the
device and keeps the fastest in a small JSON table; ``strips_for`` maps the
images of a batch to strip heights from that table (or from the library's
built-in default when no table is given).

    from paper_1905_13038_amd import tune, BatchPlan
    table = tune.autotune()                     # measures; cached on disk
    plan = BatchPlan(images, params, strips=tune.strips_for(params, table))
"""
from __future__ import annotations

import json
import os

import torch

# window-size classes (upper bounds of h) and candidate strip heights
WINDOW_CLASSES = (15, 31, 63, 127, 257)
CANDIDATES = (16, 24, 32, 48, 64, 96, 128, 192)

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1905_13038_amd",
                              "batch_strips.json")


def window_class(h: int) -> int:
    """The smallest class bound >= h (the last class for larger windows)."""
    for c in WINDOW_CLASSES:
        if h <= c:
            return c
    return WINDOW_CLASSES[-1]


def default_strip(h: int) -> int:
    """The library's default for a window of h rows: 2h, within [32, 128]."""
    return int(min(max(2 * h, 32), 128))


def strips_for(params, table=None):
    """Strip heights for a batch: one per parameter dict (key "h").  ``table``
    maps window classes (as ints or strings) to strips; missing classes use
    the default."""
    out = []
    for p in params:
        h = int(p["h"])
        s = None
        if table:
            c = window_class(h)
            s = table.get(c, table.get(str(c)))
        out.append(int(s) if s else default_strip(h))
    return out


def _synthetic_batch(count, H, W, h, seed, device):
    """`count` seeded noisy pages (uniform gray levels; timing only)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    imgs = [torch.randint(0, 256, (H, W), dtype=torch.uint8, generator=g).to(device) for _ in range(count)]
    params = [{"h": h, "w": h, "k": 0.3, "R": 128.0, "method": "sauvola"} for _ in range(count)]
    return imgs, params


def _time_plan(plan, reps):
    plan.run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def autotune(count: int = 64, H: int = 1536, W: int = 1536, candidates=CANDIDATES,
             classes=WINDOW_CLASSES, reps: int = 5, cache_path: str | None = _DEFAULT_CACHE,
             refresh: bool = False, device=None):
    """Measure the candidate strips for each window class on a batch of
    ``count`` H x W pages and return {class: best strip}.  The table is read
    from / written to ``cache_path`` (keyed by the device name) unless it is
    None; ``refresh`` forces new measurements."""
    from . import BatchPlan

    device = torch.device(device or "cuda")
    name = torch.cuda.get_device_name(device)
    cache = {}
    if cache_path and os.path.exists(cache_path) and not refresh:
        with open(cache_path) as f:
            cache = json.load(f)
        if name in cache:
            return {int(k): int(v) for k, v in cache[name].items()}
    table = {}
    for c in classes:
        h = c if c % 2 else c - 1  # an odd window at the top of the class
        h = min(h, min(H, W))
        imgs, params = _synthetic_batch(count, H, W, h, seed=c, device=device)
        times = {}
        for s in candidates:
            plan = BatchPlan(imgs, params, strips=[s] * count)
            times[s] = _time_plan(plan, reps)
            del plan
        table[c] = int(min(times, key=times.get))
        del imgs
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[name] = {str(k): v for k, v in table.items()}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return table


__all__ = ["autotune", "strips_for", "window_class", "default_strip", "WINDOW_CLASSES", "CANDIDATES"]
