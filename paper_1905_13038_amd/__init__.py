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

import torch

__all__ = [
    "lib", "BZError", "window_sums", "window_mean_std", "sauvola", "niblack",
    "window_quantile", "sauvola_batched", "BatchPlan", "soft_sauvola", "SoftSauvola",
    "LIB_PATH",
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


def window_sums(img: torch.Tensor, h: int, w: int):
    """Exact window sums S1 = sum I, S2 = sum I^2 (uint32 values held in int32
    tensors; view them as unsigned).  Returns (S1, S2)."""
    img, H, W, ld = _image(img)
    S1 = torch.empty((H, W), dtype=torch.int32, device=img.device)
    S2 = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _check(lib.bz_window_sums(img.data_ptr(), H, W, ld, h, w, S1.data_ptr(), S2.data_ptr(), W,
                              _stream(img)), "bz_window_sums")
    return S1, S2


def window_mean_std(img: torch.Tensor, h: int, w: int):
    """Window mean and population standard deviation (float32)."""
    img, H, W, ld = _image(img)
    m = torch.empty((H, W), dtype=torch.float32, device=img.device)
    s = torch.empty((H, W), dtype=torch.float32, device=img.device)
    _check(lib.bz_window_mean_std(img.data_ptr(), H, W, ld, h, w, m.data_ptr(), s.data_ptr(), W,
                                  _stream(img)), "bz_window_mean_std")
    return m, s


def _outputs(img, H, W, stats, mask, mean, std):
    if mask is None:
        mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    if stats:
        if mean is None:
            mean = torch.empty((H, W), dtype=torch.float32, device=img.device)
        if std is None:
            std = torch.empty((H, W), dtype=torch.float32, device=img.device)
    return mask, mean, std


def sauvola(img: torch.Tensor, h: int, w: int, k: float = 0.5, R: float = 128.0,
            stats: bool = True, mask=None, mean=None, std=None):
    """Sauvola mask (1 where I < m (1 + k (s/R - 1))); with ``stats`` also the
    float32 window mean and standard deviation.  Returns (mask, mean, std)."""
    img, H, W, ld = _image(img)
    mask, mean, std = _outputs(img, H, W, stats, mask, mean, std)
    ld_ms = mean.stride(0) if mean is not None else 0
    _check(lib.bz_sauvola(img.data_ptr(), H, W, ld, h, w, float(k), float(R), mask.data_ptr(),
                          mask.stride(0), mean.data_ptr() if mean is not None else None,
                          std.data_ptr() if std is not None else None, ld_ms, _stream(img)),
           "bz_sauvola")
    return mask, mean, std


def niblack(img: torch.Tensor, h: int, w: int, k: float = -0.2, stats: bool = True,
            mask=None, mean=None, std=None):
    """Niblack mask (1 where I < m + k s); returns (mask, mean, std)."""
    img, H, W, ld = _image(img)
    mask, mean, std = _outputs(img, H, W, stats, mask, mean, std)
    ld_ms = mean.stride(0) if mean is not None else 0
    _check(lib.bz_niblack(img.data_ptr(), H, W, ld, h, w, float(k), mask.data_ptr(),
                          mask.stride(0), mean.data_ptr() if mean is not None else None,
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
