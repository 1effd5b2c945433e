"""Python binding of libbinarize (gfx950 HIP kernels behind a C ABI).

Argument marshalling only: every function here validates tensor shapes,
allocates outputs with torch (device memory), and calls the matching
``bz_*`` entry point of ``libbinarize.so`` on torch's current HIP stream.
All arithmetic runs in the HIP kernels; there is no CPU fallback.  If the
library is missing, importing this package raises.

Inputs are 2-D CUDA (HIP) tensors with unit column stride; the row stride is
taken from ``tensor.stride(0)``.  See ``include/binarize.h`` for the exact
semantics of each call.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

__all__ = [
    "lib", "BZError", "window_sums", "window_mean_std", "sauvola", "niblack",
    "window_quantile", "sauvola_batched", "BatchPlan", "soft_sauvola", "SoftSauvola", "soft_window_sums",
    "global_stats", "read_global_stats", "table1_threshold", "TABLE1", "window_minmax", "bernsen",
    "binarize_streamed", "haar_features", "HAAR", "LIB_PATH", "set_tile_table",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbinarize.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libbinarize.so is not built; run `python -m paper_1905_13038_amd.build`")

_P = ctypes.c_void_p
_I = ctypes.c_int
_PD = ctypes.c_ssize_t
_F = ctypes.c_float
_D = ctypes.c_double
_SZ = ctypes.c_size_t

lib = ctypes.CDLL(LIB_PATH)
lib.bz_status_string.restype = ctypes.c_char_p
lib.bz_status_string.argtypes = [_I]
lib.bz_version.restype = _I
lib.bz_version.argtypes = []
lib.bz_max_window.restype = _I
lib.bz_max_window.argtypes = []
lib.bz_window_sums.restype = _I
lib.bz_window_sums.argtypes = [_P, _I, _I, _PD, _I, _I, _P, _P, _PD, _P]
lib.bz_window_mean_std.restype = _I
lib.bz_window_mean_std.argtypes = [_P, _I, _I, _PD, _I, _I, _P, _P, _PD, _P]
lib.bz_sauvola.restype = _I
lib.bz_sauvola.argtypes = [_P, _I, _I, _PD, _I, _I, _F, _F, _P, _PD, _P, _P, _PD, _P]
lib.bz_niblack.restype = _I
lib.bz_niblack.argtypes = [_P, _I, _I, _PD, _I, _I, _F, _P, _PD, _P, _P, _PD, _P]
lib.bz_window_quantile.restype = _I
lib.bz_window_quantile.argtypes = [_P, _I, _I, _PD, _I, _I, _D, _P, _PD, _P, _PD, _P]
lib.bz_extremes_workspace_size.restype = _SZ
lib.bz_extremes_workspace_size.argtypes = [_I, _I]
lib.bz_window_minmax.restype = _I
lib.bz_window_minmax.argtypes = [_P, _I, _I, _PD, _I, _I, _P, _P, _PD, _P, _SZ, _P]
lib.bz_bernsen.restype = _I
lib.bz_bernsen.argtypes = [_P, _I, _I, _PD, _I, _I, _I, _P, _PD, _P, _P, _PD, _P, _SZ, _P]
lib.bz_bernsen_noalloc.restype = _I
lib.bz_bernsen_noalloc.argtypes = [_P, _I, _I, _PD, _I, _I, _I, _P, _PD, _P, _P, _PD, _P]
lib.bz_bernsen_noalloc_max_pixels.restype = _SZ
lib.bz_bernsen_noalloc_max_pixels.argtypes = []
lib.bz_global_stats.restype = _I
lib.bz_global_stats.argtypes = [_P, _I, _I, _PD, _P, _P]
lib.bz_threshold.restype = _I
lib.bz_threshold.argtypes = [_P, _I, _I, _PD, _I, _I, _I, _P, _P, _P, _PD, _P, _P, _PD, _P]


class bz_item(ctypes.Structure):
    """Mirror of the C ``bz_item`` descriptor."""
    _fields_ = [("I", _P), ("mask", _P), ("mean", _P), ("std", _P),
                ("H", _I), ("W", _I), ("h", _I), ("w", _I),
                ("ld_I", _PD), ("ld_mask", _PD), ("ld_ms", _PD),
                ("k", _F), ("R", _F), ("method", _I)]


lib.bz_stream_workspace_size.restype = _SZ
lib.bz_stream_workspace_size.argtypes = [_I, _I, _I, _I, _I, _I]
lib.bz_binarize_streamed.restype = _I
lib.bz_binarize_streamed.argtypes = [_P, _I, _I, _PD, _I, _I, _I, _F, _F, _P, _PD, _I, _I, _P, _SZ, _P, _P, _P]
lib.bz_haar_workspace_size.restype = _SZ
lib.bz_haar_workspace_size.argtypes = [_I, _I, _I, _I]
lib.bz_haar_features.restype = _I
lib.bz_haar_features.argtypes = [_P, _I, _I, _PD, _I, _I, _I, _P, _PD, _P, _SZ, _P]
lib.bz_set_tile_table.restype = _I
lib.bz_set_tile_table.argtypes = [ctypes.POINTER(_I), _I]
lib.bz_batched_workspace_size.restype = _SZ
lib.bz_batched_workspace_size.argtypes = [_I]
lib.bz_batched_plan.restype = _I
lib.bz_batched_plan.argtypes = [ctypes.POINTER(bz_item), _I, ctypes.POINTER(_I), _P, _SZ, _P]
lib.bz_batched_run.restype = _I
lib.bz_batched_run.argtypes = [_P, _P]
lib.bz_sauvola_batched.restype = _I
lib.bz_sauvola_batched.argtypes = [ctypes.POINTER(bz_item), _I, _P, _SZ, _P]

METHOD_SAUVOLA, METHOD_NIBLACK = 1, 2

lib.bz_soft_workspace_size.restype = _SZ
lib.bz_soft_workspace_size.argtypes = [_I, _I, _I]
lib.bz_soft_sauvola_fwd.restype = _I
lib.bz_soft_sauvola_fwd.argtypes = [_P, _I, _I, _I, _PD, _I, _I, _P, _P, _F, _P, _P]
lib.bz_soft_window_sums.restype = _I
lib.bz_soft_window_sums.argtypes = [_P, _I, _I, _I, _PD, _I, _I, _P, _P, _PD, _P]
lib.bz_soft_sauvola_bwd.restype = _I
lib.bz_soft_sauvola_bwd.argtypes = [_P, _P, _I, _I, _I, _PD, _I, _I, _P, _P, _F, _P, _P, _P, _P,
                                    _SZ, _P]

BZ_OK, BZ_ERR_INVALID, BZ_ERR_RANGE, BZ_ERR_ALIAS, BZ_ERR_WORKSPACE, BZ_ERR_HIP = range(6)


class BZError(RuntimeError):
    """A non-OK status from libbinarize."""

    def __init__(self, status: int, fn: str):
        self.status = status
        super().__init__("%s failed: %s" % (fn, lib.bz_status_string(status).decode()))


def _check(status: int, fn: str):
    if status != BZ_OK:
        if status in (BZ_ERR_INVALID, BZ_ERR_RANGE, BZ_ERR_ALIAS, BZ_ERR_WORKSPACE):
            raise ValueError(str(BZError(status, fn)))
        raise BZError(status, fn)


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _image(img: torch.Tensor, dtype=torch.uint8):
    if not isinstance(img, torch.Tensor) or img.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if img.dtype != dtype:
        raise ValueError("expected dtype %s" % dtype)
    if not img.is_cuda:
        raise ValueError("expected a device (HIP) tensor; there is no CPU path")
    if img.stride(1) != 1:
        img = img.contiguous()
    H, W = img.shape
    ld = img.stride(0) if H > 1 else W
    return img, H, W, max(ld, W)


def set_tile_table(rows):
    """Install the tiling table of the single-image calls: rows of (largest h,
    largest W, strip rows, threads), e.g. from ``tune.autotune_plain``; an
    empty list removes it (``bz_set_tile_table``)."""
    flat = [int(v) for r in rows for v in r]
    if len(flat) != 4 * len(rows):
        raise ValueError("each row holds four ints")
    arr = (_I * max(len(flat), 1))(*flat)
    _check(lib.bz_set_tile_table(ctypes.cast(arr, ctypes.POINTER(_I)), len(rows)), "bz_set_tile_table")


_tiling_done = False


def _tiling():
    """On the first single-image call of the process: unless BZ_TILE_S or
    BZ_TILE_THREADS is set, install the autotuner's cached table for this
    device, if there is a readable one (a missing or corrupt cache leaves the
    built-in plan)."""
    global _tiling_done
    if _tiling_done:
        return
    _tiling_done = True
    if os.environ.get("BZ_TILE_S") or os.environ.get("BZ_TILE_THREADS"):
        return
    from . import tune
    rows = tune.cached_plain_rows()
    if rows:
        set_tile_table(rows)


def window_sums(img: torch.Tensor, h: int, w: int):
    """Exact window sums S1 = sum I, S2 = sum I^2 (uint32 values held in int32
    tensors; view them as unsigned).  Returns (S1, S2)."""
    _tiling()
    img, H, W, ld = _image(img)
    S1 = torch.empty((H, W), dtype=torch.int32, device=img.device)
    S2 = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _check(lib.bz_window_sums(img.data_ptr(), H, W, ld, h, w, S1.data_ptr(), S2.data_ptr(), W,
                              _stream(img)), "bz_window_sums")
    return S1, S2


def window_mean_std(img: torch.Tensor, h: int, w: int):
    """Window mean and population standard deviation (float32)."""
    _tiling()
    img, H, W, ld = _image(img)
    m = torch.empty((H, W), dtype=torch.float32, device=img.device)
    s = torch.empty((H, W), dtype=torch.float32, device=img.device)
    _check(lib.bz_window_mean_std(img.data_ptr(), H, W, ld, h, w, m.data_ptr(), s.data_ptr(), W,
                                  _stream(img)), "bz_window_mean_std")
    return m, s


def _given_output(t, name, H, W, dtype, device):
    """A caller-provided output: the kernels write H rows of W elements at
    row stride t.stride(0), so shape, dtype, device and unit column stride
    must match exactly."""
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device:
        raise ValueError("%s must be a %s tensor on %s" % (name, dtype, device))
    if tuple(t.shape) != (H, W) or (W > 1 and t.stride(1) != 1) or (H > 1 and t.stride(0) < W):
        raise ValueError("%s must have shape (%d, %d) with unit column stride" % (name, H, W))
    return t


def _outputs(img, H, W, stats, mask, mean, std):
    if mask is None:
        mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    else:
        _given_output(mask, "mask", H, W, torch.uint8, img.device)
    if not stats:
        if mean is not None or std is not None:
            raise ValueError("mean/std outputs given with stats=False")
        return mask, None, None
    for t, name in ((mean, "mean"), (std, "std")):
        if t is not None:
            _given_output(t, name, H, W, torch.float32, img.device)
    # mean and std share one row stride (the C ABI takes one ld for both)
    ref = mean if mean is not None else std
    ld_ms = _ld(ref, W) if ref is not None else W
    if mean is None:
        mean = torch.empty_strided((H, W), (ld_ms, 1), dtype=torch.float32, device=img.device)
    if std is None:
        std = torch.empty_strided((H, W), (ld_ms, 1), dtype=torch.float32, device=img.device)
    if _ld(mean, W) != _ld(std, W):
        raise ValueError("mean and std must share one row stride")
    return mask, mean, std


def _ld(t, W):
    """Row stride of an output for the C ABI (W for a single row)."""
    return t.stride(0) if t.shape[0] > 1 else W


def sauvola(img: torch.Tensor, h: int, w: int, k: float = 0.5, R: float = 128.0,
            stats: bool = True, mask=None, mean=None, std=None):
    """Sauvola mask (1 where I < m (1 + k (s/R - 1))); with ``stats`` also the
    float32 window mean and standard deviation.  Returns (mask, mean, std)."""
    _tiling()
    img, H, W, ld = _image(img)
    mask, mean, std = _outputs(img, H, W, stats, mask, mean, std)
    ld_ms = _ld(mean, W) if mean is not None else 0
    _check(lib.bz_sauvola(img.data_ptr(), H, W, ld, h, w, float(k), float(R), mask.data_ptr(),
                          _ld(mask, W), mean.data_ptr() if mean is not None else None,
                          std.data_ptr() if std is not None else None, ld_ms, _stream(img)),
           "bz_sauvola")
    return mask, mean, std


def niblack(img: torch.Tensor, h: int, w: int, k: float = -0.2, stats: bool = True,
            mask=None, mean=None, std=None):
    """Niblack mask (1 where I < m + k s); returns (mask, mean, std)."""
    _tiling()
    img, H, W, ld = _image(img)
    mask, mean, std = _outputs(img, H, W, stats, mask, mean, std)
    ld_ms = _ld(mean, W) if mean is not None else 0
    _check(lib.bz_niblack(img.data_ptr(), H, W, ld, h, w, float(k), mask.data_ptr(),
                          _ld(mask, W), mean.data_ptr() if mean is not None else None,
                          std.data_ptr() if std is not None else None, ld_ms, _stream(img)),
           "bz_niblack")
    return mask, mean, std


def window_quantile(img: torch.Tensor, h: int, w: int, q: float, with_mask: bool = True):
    """Windowed q-quantile (rho-th smallest, rho = max(1, ceil(q n))) and the
    mask I < Q.  Returns (Q, mask or None)."""
    img, H, W, ld = _image(img)
    Q = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    mask = torch.empty((H, W), dtype=torch.uint8, device=img.device) if with_mask else None
    _check(lib.bz_window_quantile(img.data_ptr(), H, W, ld, h, w, float(q), Q.data_ptr(), W,
                                  mask.data_ptr() if mask is not None else None, W,
                                  _stream(img)), "bz_window_quantile")
    return Q, mask


class BatchPlan:
    """A planned ragged batch: every image gets its own outputs, window and
    parameters; ``run()`` binarizes all of them in ONE persistent kernel
    launch, and ``capture()`` records that launch in a HIP graph for replay.

    images: list of 2-D uint8 device tensors.  params: list of dicts with keys
    h, w, k, R (optional, default 128), method ("sauvola" or "niblack"), stats
    (optional bool, default True: also write mean/std).  strips: optional list
    of per-image strip heights (rows), e.g. from ``tune.strips_for``.

    The outputs are (H, W) views of row-padded storage: every mask row and
    every mean/std row starts on a 64-byte boundary (pitch W rounded up to 64
    bytes and to 16 floats), so a wavefront's stores never straddle two
    64-byte segments of a row.
    """

    def __init__(self, images, params, strips=None):
        if len(images) != len(params) or not images:
            raise ValueError("need one parameter dict per image")
        dev = images[0].device
        self.images, self.masks, self.means, self.stds = [], [], [], []
        items = (bz_item * len(images))()
        for i, (img, p) in enumerate(zip(images, params)):
            img, H, W, ld = _image(img)
            if img.device != dev:
                raise ValueError("all images must be on one device")
            self.images.append(img)
            ld_mask = -(-W // 64) * 64
            ld_ms = -(-W // 16) * 16
            mask = torch.empty((H, ld_mask), dtype=torch.uint8, device=dev)[:, :W]
            stats = p.get("stats", True)
            mean = torch.empty((H, ld_ms), dtype=torch.float32, device=dev)[:, :W] if stats else None
            std = torch.empty((H, ld_ms), dtype=torch.float32, device=dev)[:, :W] if stats else None
            self.masks.append(mask)
            self.means.append(mean)
            self.stds.append(std)
            method = p.get("method", "sauvola")
            items[i] = bz_item(img.data_ptr(), mask.data_ptr(),
                               mean.data_ptr() if mean is not None else None,
                               std.data_ptr() if std is not None else None,
                               H, W, int(p["h"]), int(p["w"]), ld, ld_mask, ld_ms if stats else 0,
                               float(p["k"]), float(p.get("R", 128.0)),
                               METHOD_SAUVOLA if method == "sauvola" else METHOD_NIBLACK)
        self._items = items
        n = len(images)
        self.ws_bytes = int(lib.bz_batched_workspace_size(n))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.replan(strips)

    def replan(self, strips=None):
        """Plan the same images and outputs again with other strip heights
        (None: the library's defaults); a captured graph is dropped."""
        n = len(self.images)
        if strips is not None:
            arr = (_I * n)(*[int(x) for x in strips])
            sp = ctypes.cast(arr, ctypes.POINTER(_I))
        else:
            sp = None
        _check(lib.bz_batched_plan(self._items, n, sp, self.workspace.data_ptr(), self.ws_bytes,
                                   _stream(self.workspace)), "bz_batched_plan")
        self.graph = None

    def run(self):
        """Enqueue the persistent launch on the current stream."""
        _check(lib.bz_batched_run(self.workspace.data_ptr(), _stream(self.workspace)),
               "bz_batched_run")

    def capture(self):
        """Record ``run()`` in a HIP graph (torch.cuda.CUDAGraph); later calls
        to ``replay()`` launch it without host-side work."""
        self.run()  # warm up the launch path outside capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def outputs(self):
        return list(zip(self.masks, self.means, self.stds))


def sauvola_batched(images, params, strips=None):
    """One-shot ragged batch: plan, run once, return [(mask, mean, std), ...]."""
    plan = BatchPlan(images, params, strips)
    plan.run()
    return plan.outputs()


def window_minmax(img: torch.Tensor, h: int, w: int):
    """Minimum and maximum of each pixel's clipped window (uint8, exact).
    Returns (mn, mx)."""
    img, H, W, ld = _image(img)
    mn = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    mx = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    nb = int(lib.bz_extremes_workspace_size(H, W))
    ws = torch.empty(nb, dtype=torch.uint8, device=img.device)
    _check(lib.bz_window_minmax(img.data_ptr(), H, W, ld, h, w, mn.data_ptr(), mx.data_ptr(), W,
                                ws.data_ptr(), nb, _stream(img)), "bz_window_minmax")
    return mn, mx


def bernsen(img: torch.Tensor, h: int, w: int, contrast_min: int = 15):
    """Bernsen's midrange rule: mask = 1 where the window's range reaches
    ``contrast_min`` and 2 I < min + max.  Returns (mask, mn, mx)."""
    img, H, W, ld = _image(img)
    mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    mn = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    mx = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    nb = int(lib.bz_extremes_workspace_size(H, W))
    ws = torch.empty(nb, dtype=torch.uint8, device=img.device)
    _check(lib.bz_bernsen(img.data_ptr(), H, W, ld, h, w, int(contrast_min), mask.data_ptr(), W,
                          mn.data_ptr(), mx.data_ptr(), W, ws.data_ptr(), nb, _stream(img)), "bz_bernsen")
    return mask, mn, mx


# Haar-like feature templates: C-ABI code and cell grid (rows, columns)
HAAR = {"edge_h": (1, (1, 2)), "edge_v": (2, (2, 1)), "line_h": (3, (1, 3)), "line_v": (4, (3, 1)),
        "checker": (5, (2, 2))}


def haar_features(img: torch.Tensor, a: int, b: int, kind: str) -> torch.Tensor:
    """Haar-like feature ``kind`` (a key of HAAR) with cells of a rows by b
    columns at every anchor where the template fits: an int32 tensor of
    (H - kv a + 1) x (W - kh b + 1)."""
    if kind not in HAAR:
        raise ValueError("kind must be one of %s" % sorted(HAAR))
    img, H, W, ld = _image(img)
    code, (kv, kh) = HAAR[kind]
    Hf, Wf = H - kv * a + 1, W - kh * b + 1
    if Hf < 1 or Wf < 1:
        raise ValueError("the template does not fit in the image")
    F = torch.empty((Hf, Wf), dtype=torch.int32, device=img.device)
    nb = int(lib.bz_haar_workspace_size(H, W, a, code))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=img.device)
    _check(lib.bz_haar_features(img.data_ptr(), H, W, ld, a, b, code, F.data_ptr(), Wf, ws.data_ptr(), nb,
                                _stream(img)), "bz_haar_features")
    return F


_STREAM_METHODS = {"sauvola": 1, "niblack": 2}
_AXES = {"auto": 0, "rows": 1, "columns": 2}
_copy_streams = {}


def _host_image(img, name):
    if not isinstance(img, torch.Tensor) or img.dim() != 2 or img.dtype != torch.uint8:
        raise ValueError("%s: expected a 2-D uint8 tensor" % name)
    if img.is_cuda:
        raise ValueError("%s: expected a host (CPU) tensor" % name)
    if img.stride(1) != 1:
        raise ValueError("%s: expected unit column stride" % name)
    H, W = img.shape
    return max(img.stride(0) if H > 1 else W, W)


def binarize_streamed(img: torch.Tensor, h: int, w: int, method: str = "sauvola", k: float = 0.5,
                      R: float = 128.0, out: torch.Tensor = None, band: int = None, axis: str = "auto",
                      device=None):
    """Sauvola or Niblack over a HOST (CPU) uint8 image, streamed through the
    device in bands of rows or columns (``axis``: "rows", "columns" or
    "auto", which takes rows where they fit) with the window's halo; returns
    when the mask is complete.  ``out``: the CPU uint8 tensor for the mask,
    which may be ``img`` itself (in-place binarization); by default a new
    tensor, page-locked when ``img`` is.  ``band``: lines per band (default:
    device slots of about 32 MiB).  Returns the mask."""
    if method not in _STREAM_METHODS:
        raise ValueError("method must be 'sauvola' or 'niblack'")
    if axis not in _AXES:
        raise ValueError("axis must be 'auto', 'rows' or 'columns'")
    _tiling()
    ld = _host_image(img, "img")
    H, W = img.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, pin_memory=img.is_pinned())
    if tuple(out.shape) != (H, W):
        raise ValueError("out: expected shape %s" % ((H, W),))
    ld_out = _host_image(out, "out")
    if band is None:
        rows = axis == "rows" or (axis == "auto" and (h + 1) * (-(-W // 64) * 64) < (1 << 31))
        cross, win = (W, h) if rows else (H, w)
        band = max(1, max(64, (1 << 25) // max(cross, 1)) - (win - 1))
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    nb = int(lib.bz_stream_workspace_size(H, W, h, w, int(band), _AXES[axis]))
    if nb == 0:
        _check(BZ_ERR_INVALID, "bz_stream_workspace_size")
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    if dev not in _copy_streams:  # default priority, one pair per device
        _copy_streams[dev] = (torch.cuda.Stream(dev), torch.cuda.Stream(dev))
    load, store = _copy_streams[dev]
    with torch.cuda.device(dev):
        cs = torch.cuda.current_stream(dev).cuda_stream
        _check(lib.bz_binarize_streamed(img.data_ptr(), H, W, ld, h, w, _STREAM_METHODS[method], k, R,
                                        out.data_ptr(), ld_out, int(band), _AXES[axis], ws.data_ptr(), nb,
                                        ctypes.c_void_p(cs), ctypes.c_void_p(load.cuda_stream),
                                        ctypes.c_void_p(store.cuda_stream)),
               "bz_binarize_streamed")
    return out


# The other rules of Table 1: C-ABI code and parameter names, in order.
TABLE1 = {
    "wolf": (3, ("k", "R")),
    "feng": (4, ("a1", "k1", "k2", "gamma", "R")),
    "rais": (5, ()),
    "nick": (6, ("k",)),
    "phansalkar": (7, ("p", "q", "k", "R")),
}
_NEEDS_GLOBAL = {"wolf", "feng", "rais"}
GLOBAL_DTYPE = np.dtype([("n", "<u8"), ("sum", "<u8"), ("sumsq", "<u8"), ("min", "<u4"),
                         ("max", "<u4"), ("mean", "<f8"), ("std", "<f8")])


def global_stats(img: torch.Tensor) -> torch.Tensor:
    """Table 1's global statistics (minimum L, mean M, standard deviation S,
    with the exact sums) of a uint8 device image, as the 48-byte device record
    bz_global; read it on the host with ``read_global_stats``."""
    img, H, W, ld = _image(img)
    rec = torch.empty(GLOBAL_DTYPE.itemsize, dtype=torch.uint8, device=img.device)
    _check(lib.bz_global_stats(img.data_ptr(), H, W, ld, rec.data_ptr(), _stream(img)),
           "bz_global_stats")
    return rec


def read_global_stats(rec: torch.Tensor) -> dict:
    """The fields of a bz_global record (copies it to the host)."""
    a = rec.cpu().numpy().view(GLOBAL_DTYPE)[0]
    return {k: a[k].item() for k in GLOBAL_DTYPE.names}


def table1_threshold(img: torch.Tensor, h: int, w: int, method: str, params=None, stats=None,
                     with_stats: bool = True, mask=None, mean=None, std=None):
    """Wolf, Feng, Rais, Khurshid (NICK) or Phansalkar thresholding (Table 1):
    mask = 1 where I < t, decided in binary64.  ``params``: dict or sequence
    in the order of ``TABLE1[method][1]`` (Rais takes none).  ``stats``: the
    image's global-statistics record; computed here when the rule needs it and
    none is given.  Returns (mask, mean, std)."""
    if method not in TABLE1:
        raise ValueError("method must be one of %s" % ", ".join(TABLE1))
    code, names = TABLE1[method]
    if isinstance(params, dict):
        vals = [float(params[n]) for n in names]
    else:
        vals = [float(v) for v in (params or ())]
    if len(vals) != len(names):
        raise ValueError("%s takes parameters %s" % (method, names))
    _tiling()
    img, H, W, ld = _image(img)
    if method in _NEEDS_GLOBAL and stats is None:
        stats = global_stats(img)
    if stats is not None and (not isinstance(stats, torch.Tensor) or stats.device != img.device
                              or stats.dtype != torch.uint8 or stats.numel() != GLOBAL_DTYPE.itemsize
                              or not stats.is_contiguous()):
        raise ValueError("stats must be a 48-byte uint8 record on the image's device")
    mask, mean, std = _outputs(img, H, W, with_stats, mask, mean, std)
    ld_ms = _ld(mean, W) if mean is not None else 0
    pv = (ctypes.c_double * 5)(*(vals + [0.0] * (5 - len(vals))))
    _check(lib.bz_threshold(img.data_ptr(), H, W, ld, h, w, code, pv,
                            stats.data_ptr() if stats is not None else None, mask.data_ptr(),
                            _ld(mask, W), mean.data_ptr() if mean is not None else None,
                            std.data_ptr() if std is not None else None, ld_ms, _stream(img)),
           "bz_threshold")
    return mask, mean, std


def _soft_inputs(I, k, R):
    if I.dim() == 2:
        I = I.unsqueeze(0)
    if I.dim() != 3 or I.dtype != torch.float32 or not I.is_cuda:
        raise ValueError("expected a (B, H, W) float32 device tensor")
    I = I.contiguous()
    B, H, W = I.shape
    k = k.reshape(-1).to(torch.float32).contiguous()
    R = R.reshape(-1).to(torch.float32).contiguous()
    if k.numel() != B or R.numel() != 1 or not k.is_cuda or not R.is_cuda:
        raise ValueError("k must hold B values and R one value, on the device")
    return I, k, R, B, H, W


class SoftSauvola(torch.autograd.Function):
    """y = sigmoid((I - t) / tau) with the Sauvola threshold t of each pixel's
    window; differentiable in I, k (one per image) and R.  Only I, k and R are
    saved: the backward recomputes the window statistics."""

    @staticmethod
    def forward(ctx, I, k, R, h, w, tau):
        shapes = (I.shape, k.shape, R.shape)
        I, k, R, B, H, W = _soft_inputs(I, k, R)
        y = torch.empty_like(I)
        _check(lib.bz_soft_sauvola_fwd(I.data_ptr(), B, H, W, W, int(h), int(w), k.data_ptr(),
                                       R.data_ptr(), float(tau), y.data_ptr(), _stream(I)),
               "bz_soft_sauvola_fwd")
        ctx.save_for_backward(I, k, R)
        ctx.win = (int(h), int(w), float(tau))
        ctx.shapes = shapes
        return y.reshape(shapes[0])

    @staticmethod
    def backward(ctx, gy):
        I, k, R = ctx.saved_tensors
        h, w, tau = ctx.win
        B, H, W = I.shape
        gy = gy.reshape(B, H, W).to(torch.float32).contiguous()
        gI = torch.empty_like(I)
        gk = torch.empty_like(k)
        gR = torch.empty_like(R)
        nbytes = int(lib.bz_soft_workspace_size(B, H, W))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=I.device)
        _check(lib.bz_soft_sauvola_bwd(I.data_ptr(), gy.data_ptr(), B, H, W, W, h, w, k.data_ptr(),
                                       R.data_ptr(), float(tau), gI.data_ptr(), gk.data_ptr(),
                                       gR.data_ptr(), ws.data_ptr(), nbytes, _stream(I)),
               "bz_soft_sauvola_bwd")
        # gradients in the shapes the caller passed (k may be (B, 1), R 0-d)
        sI, sk, sR = ctx.shapes
        return gI.reshape(sI), gk.reshape(sk), gR.reshape(sR), None, None, None


def soft_window_sums(I: torch.Tensor, h: int, w: int):
    """The binary64 window sums (S1, S2) the soft calls compute, for a (B, H, W)
    or (H, W) float32 device tensor (test export of the running sums)."""
    if I.dim() == 2:
        I = I.unsqueeze(0)
    if I.dim() != 3 or I.dtype != torch.float32 or not I.is_cuda:
        raise ValueError("expected a (B, H, W) float32 device tensor")
    I = I.contiguous()
    B, H, W = I.shape
    S1 = torch.empty((B, H, W), dtype=torch.float64, device=I.device)
    S2 = torch.empty_like(S1)
    _check(lib.bz_soft_window_sums(I.data_ptr(), B, H, W, W, int(h), int(w), S1.data_ptr(), S2.data_ptr(), W,
                                   _stream(I)), "bz_soft_window_sums")
    return S1, S2


def soft_sauvola(I, k, R, h: int, w: int, tau: float = 2.0):
    """Differentiable soft Sauvola mask of a (B, H, W) float32 stack."""
    return SoftSauvola.apply(I, k, R, h, w, tau)
