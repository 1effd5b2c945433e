"""Autotuner of the tilings: strip heights of ragged batches, and strip
heights and block sizes of single-image calls.

A batched launch processes each image in tiles of one strip of rows; every
strip first primes its column sums over the h - 1 rows above and below its
first row, so short strips waste priming work and tall strips leave fewer
tiles to balance across the persistent grid.  ``autotune`` measures, per
window-size class, the batch time of a few candidate strip heights on a
synthetic batch and caches the table; ``autotune_plan`` tunes the classes of
one planned batch on that batch itself; ``strips_for`` maps the images of a
batch to strip heights from a table (or from the library's built-in default
when no table is given).

A single-image call runs one tile per strip of rows and block of columns;
``autotune_plain`` measures, per window-size class and width class, candidate
strip heights and block sizes (through the BZ_TILE_S / BZ_TILE_THREADS
overrides) and returns rows (largest h, largest W, strip, threads) for
``bz_set_tile_table``.  The binding installs the cached rows on its first
single-image call unless BZ_TILE_S or BZ_TILE_THREADS is set.

Both tables are kept in one JSON file keyed by the device name.  A cache that
cannot be read, or whose entry for the device does not have the expected
shape, is ignored: the tuner measures again and the calls keep the built-in
plans meanwhile.

    from paper_1905_13038_amd import tune, BatchPlan, set_tile_table
    table = tune.autotune()                     # measures; cached on disk
    plan = BatchPlan(images, params, strips=tune.strips_for(params, table))
    set_tile_table(tune.autotune_plain())
"""
from __future__ import annotations

import json
import os

import torch

# window-size classes (upper bounds of h) and candidate strip heights
WINDOW_CLASSES = (15, 31, 63, 127, 257)
CANDIDATES = (16, 24, 32, 48, 64, 96, 128, 192)
# single-image calls: width classes (upper bounds of W), candidate strips and
# block sizes
WIDTH_CLASSES = (1024, 2048, 4096, 8192)
PLAIN_STRIPS = (4, 8, 12, 16, 24, 32)
PLAIN_THREADS = (256, 512, 1024)

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1905_13038_amd",
                              "tilings.json")


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


def _valid_batch(entry):
    if not isinstance(entry, dict) or not entry:
        return None
    out = {}
    for k, v in entry.items():
        c, s = int(k), int(v)
        if c < 1 or s < 1:
            return None
        out[c] = s
    return out


def _valid_plain(entry):
    if not isinstance(entry, list) or not entry:
        return None
    rows = []
    for r in entry:
        if not isinstance(r, list) or len(r) != 4:
            return None
        hmax, wmax, strip, threads = (int(v) for v in r)
        if hmax < 1 or wmax < 1 or strip < 0 or threads < 0 or threads > 1024 or threads % 64:
            return None
        rows.append([hmax, wmax, strip, threads])
    return rows


def load_table(cache_path, device_name: str, kind: str):
    """The cached table of ``kind`` ("batch": {class: strip}; "plain": rows of
    four ints) for ``device_name``, or None when the file is missing,
    unreadable, not JSON, or holds no entry of the expected shape."""
    if not cache_path or not os.path.exists(cache_path):
        return None
    try:
        with open(cache_path) as f:
            cache = json.load(f)
        entry = cache[device_name][kind]
        return _valid_batch(entry) if kind == "batch" else _valid_plain(entry)
    except (OSError, ValueError, KeyError, TypeError, AttributeError):
        return None


def save_table(cache_path, device_name: str, kind: str, table) -> None:
    """Store ``table`` under (device, kind), keeping the file's other entries
    when it is readable (a corrupt file is replaced)."""
    cache = {}
    if os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
            if not isinstance(cache, dict):
                cache = {}
        except (OSError, ValueError):
            cache = {}
    dev = cache.get(device_name)
    if not isinstance(dev, dict):
        dev = {}
    dev[kind] = ({str(k): int(v) for k, v in table.items()} if kind == "batch"
                 else [[int(v) for v in r] for r in table])
    cache[device_name] = dev
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    tmp = cache_path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)


def _synthetic_batch(count, H, W, h, seed, device):
    """`count` seeded noisy pages (uniform gray levels; timing only)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    imgs = [torch.randint(0, 256, (H, W), dtype=torch.uint8, generator=g).to(device) for _ in range(count)]
    params = [{"h": h, "w": h, "k": 0.3, "R": 128.0, "method": "sauvola"} for _ in range(count)]
    return imgs, params


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
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
    if not refresh:
        cached = load_table(cache_path, name, "batch")
        if cached:
            return cached
    table = {}
    for c in classes:
        h = c if c % 2 else c - 1  # an odd window at the top of the class
        h = min(h, min(H, W))
        imgs, params = _synthetic_batch(count, H, W, h, seed=c, device=device)
        times = {}
        for s in candidates:
            plan = BatchPlan(imgs, params, strips=[s] * count)
            times[s] = _time(plan.run, reps)
            del plan
        table[c] = int(min(times, key=times.get))
        del imgs
    if cache_path:
        save_table(cache_path, name, "batch", table)
    return table


def autotune_plan(plan, params, candidates=CANDIDATES, reps: int = 5, min_gain: float = 0.005):
    """Tune the strips of one planned batch on the batch itself: starting
    from the built-in strips, each window class present takes in turn the
    candidate that makes the whole launch fastest (kept only if it gains at
    least ``min_gain``).  Leaves ``plan`` planned with the result and returns
    the table {class: strip} (classes left at the built-in strip are absent)."""
    classes = sorted(set(window_class(int(p["h"])) for p in params))
    table = {}
    plan.replan(strips_for(params, table))
    best = _time(plan.run, reps)
    for c in classes:
        pick = None
        for s in candidates:
            trial = dict(table)
            trial[c] = s
            plan.replan(strips_for(params, trial))
            t = _time(plan.run, reps)
            if t < best * (1.0 - min_gain):
                best, pick = t, s
        if pick is not None:
            table[c] = pick
    plan.replan(strips_for(params, table))
    return table


def autotune_plain(H: int = 3072, classes=WINDOW_CLASSES, widths=WIDTH_CLASSES, strips=PLAIN_STRIPS,
                   threads=PLAIN_THREADS, reps: int = 5, cache_path: str | None = _DEFAULT_CACHE,
                   refresh: bool = False, device=None):
    """Measure, for each window class and width class, Sauvola (mask, mean and
    std) on an H x (class width) page with every candidate strip and block
    size, and return the rows (largest h, largest W, best strip, best threads)
    for ``set_tile_table``, one per class; the library's built-in plan is one
    candidate, and a class where it is the fastest gets strip 0 and threads 0
    (the built-in choice)."""
    from . import sauvola

    device = torch.device(device or "cuda")
    name = torch.cuda.get_device_name(device)
    if not refresh:
        cached = load_table(cache_path, name, "plain")
        if cached:
            return cached
    saved = {k: os.environ.pop(k, None) for k in ("BZ_TILE_S", "BZ_TILE_THREADS")}
    rows = []
    try:
        g = torch.Generator(device="cpu").manual_seed(11)
        for wc in widths:
            img = torch.randint(0, 256, (H, wc), dtype=torch.uint8, generator=g).to(device)
            outs = (torch.empty((H, wc), dtype=torch.uint8, device=device),
                    torch.empty((H, wc), dtype=torch.float32, device=device),
                    torch.empty((H, wc), dtype=torch.float32, device=device))
            for c in classes:
                h = c if c % 2 else c - 1
                h = min(h, H, wc)

                def call():
                    sauvola(img, h, h, 0.5, 128.0, mask=outs[0], mean=outs[1], std=outs[2])
                os.environ.pop("BZ_TILE_S", None)
                os.environ.pop("BZ_TILE_THREADS", None)
                best = (_time(call, reps), None)
                for s in strips:
                    for t in threads:
                        os.environ["BZ_TILE_S"] = str(s)
                        os.environ["BZ_TILE_THREADS"] = str(t)
                        ms = _time(call, reps)
                        if ms < best[0]:
                            best = (ms, (s, t))
                rows.append([c, wc] + (list(best[1]) if best[1] is not None else [0, 0]))
            del img, outs
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    if cache_path and rows:
        save_table(cache_path, name, "plain", rows)
    return rows


def cached_plain_rows(cache_path: str | None = _DEFAULT_CACHE, device=None):
    """The cached single-image rows for the current device, or None (no
    measurement)."""
    if not cache_path or not os.path.exists(cache_path):
        return None
    try:
        name = torch.cuda.get_device_name(torch.device(device or "cuda"))
    except (RuntimeError, AssertionError):
        return None
    return load_table(cache_path, name, "plain")


__all__ = ["autotune", "autotune_plan", "autotune_plain", "strips_for", "window_class", "default_strip", "load_table",
           "save_table", "cached_plain_rows", "WINDOW_CLASSES", "WIDTH_CLASSES", "CANDIDATES",
           "PLAIN_STRIPS", "PLAIN_THREADS"]
