"""Torch-facing calls of the fast Haar transform (tensors in, tensors out).

PyTorch supplies device memory and the current stream only; every transform
runs in libhaar's HIP kernels.  Shapes: 1D ``[..., n]`` (leading dims are the
batch), 2D ``[..., h, w]``.  Storage dtypes: float32, bfloat16, float16.
Outputs are new contiguous tensors of the input's shape, in the packed layout
``[a_L | d_L | ... | d_1]`` (1D) or the quadrant layout (2D).
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi

DTYPE_CODES = {torch.float32: 0, torch.bfloat16: 1, torch.float16: 2}


def dtype_code(t: torch.Tensor) -> int:
    try:
        return DTYPE_CODES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32, bfloat16 or float16") from None


# The raw handle of the current stream without building a torch.cuda.Stream
# object per call (a few microseconds each, which the autograd step pays
# twice); torch.cuda.current_stream is the fallback.
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(dev) -> int:
    if _raw_stream is not None and dev.index is not None:
        return _raw_stream(dev.index)
    return torch.cuda.current_stream(dev).cuda_stream


def _prep(x: torch.Tensor, dims: int) -> torch.Tensor:
    if not x.is_cuda:
        raise ValueError("libhaar works on GPU tensors (got a CPU tensor)")
    if x.dim() < dims:
        raise ValueError(f"need at least {dims} dimension(s), got shape {tuple(x.shape)}")
    return x.contiguous()


def _out(x, out):
    if out is None:
        return torch.empty_like(x)
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the input's shape, dtype and device")
    return out


def max_levels_1d(n: int) -> int:
    return _abi.haar_max_levels_1d(n)


def max_levels_2d(h: int, w: int) -> int:
    return _abi.haar_max_levels_2d(h, w)


def fwd1d(x: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level 1D analysis along the last axis."""
    x = _prep(x, 1)
    y = _out(x, out)
    n = x.shape[-1]
    batch = x.numel() // n if n > 0 else 0
    _abi.check(_abi.haar_fwd_1d(x.data_ptr(), y.data_ptr(), n, int(levels), batch, dtype_code(x),
                                _stream(x.device)))
    return y


def inv1d(y: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level 1D synthesis along the last axis (inverse of fwd1d)."""
    y = _prep(y, 1)
    x = _out(y, out)
    n = y.shape[-1]
    batch = y.numel() // n if n > 0 else 0
    _abi.check(_abi.haar_inv_1d(y.data_ptr(), x.data_ptr(), n, int(levels), batch, dtype_code(y),
                                _stream(y.device)))
    return x


def fwd2d(x: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level separable 2D analysis on the last two axes."""
    x = _prep(x, 2)
    y = _out(x, out)
    h, w = x.shape[-2], x.shape[-1]
    batch = x.numel() // (h * w) if h * w > 0 else 0
    _abi.check(_abi.haar_fwd_2d(x.data_ptr(), y.data_ptr(), h, w, int(levels), batch, dtype_code(x),
                                _stream(x.device)))
    return y


def inv2d(y: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level separable 2D synthesis on the last two axes (inverse of fwd2d)."""
    y = _prep(y, 2)
    x = _out(y, out)
    h, w = y.shape[-2], y.shape[-1]
    batch = y.numel() // (h * w) if h * w > 0 else 0
    _abi.check(_abi.haar_inv_2d(y.data_ptr(), x.data_ptr(), h, w, int(levels), batch, dtype_code(y),
                                _stream(y.device)))
    return x


def fwd3d(x: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level separable 3D analysis on the last three axes (depth,
    height, width): x, then y, then z per level, recursion on LLL."""
    x = _prep(x, 3)
    y = _out(x, out)
    d, h, w = x.shape[-3], x.shape[-2], x.shape[-1]
    batch = x.numel() // (d * h * w) if d * h * w > 0 else 0
    _abi.check(_abi.haar_fwd_3d(x.data_ptr(), y.data_ptr(), d, h, w, int(levels), batch, dtype_code(x),
                                _stream(x.device)))
    return y


def inv3d(y: torch.Tensor, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Multi-level separable 3D synthesis on the last three axes (inverse of fwd3d)."""
    y = _prep(y, 3)
    x = _out(y, out)
    d, h, w = y.shape[-3], y.shape[-2], y.shape[-1]
    batch = y.numel() // (d * h * w) if d * h * w > 0 else 0
    _abi.check(_abi.haar_inv_3d(y.data_ptr(), x.data_ptr(), d, h, w, int(levels), batch, dtype_code(y),
                                _stream(y.device)))
    return x


def l1_grad2d(x: torch.Tensor, levels: int, out: torch.Tensor | None = None):
    """One fused pass: the loss sum |details| + 0.5 ||LL_L||^2 of the 2D
    analysis of each item of x and its gradient with respect to x.
    Returns (loss, grad): loss is a float64 tensor of the batch shape."""
    x = _prep(x, 2)
    g = _out(x, out)
    h, w = x.shape[-2], x.shape[-1]
    batch = x.numel() // (h * w) if h * w > 0 else 0
    loss = torch.empty(x.shape[:-2], dtype=torch.float64, device=x.device)
    _abi.check(_abi.haar_l1_grad_2d(x.data_ptr(), g.data_ptr(), loss.data_ptr() if batch else 0, h, w,
                                    int(levels), batch, dtype_code(x), _stream(x.device)))
    return loss, g


SHRINK_MODES = {"hard": 0, "soft": 1}


def _thresholds(levels: int, thresholds):
    if isinstance(thresholds, (int, float)):
        return [float(thresholds)] * int(levels)
    vals = [float(t) for t in thresholds]
    if len(vals) != int(levels):
        raise ValueError(f"need one threshold per level ({levels}), got {len(vals)}")
    return vals


def shrink1d(x: torch.Tensor, levels: int, thresholds, mode: str = "hard",
             out: torch.Tensor | None = None) -> torch.Tensor:
    """Fused analysis -> thresholding of the level-j details with thresholds[j-1]
    (one float applies to every level) -> synthesis, along the last axis."""
    x = _prep(x, 1)
    y = _out(x, out)
    n = x.shape[-1]
    batch = x.numel() // n if n > 0 else 0
    _abi.check(_abi.haar_shrink_1d(x.data_ptr(), y.data_ptr(), n, int(levels), batch, dtype_code(x),
                                   SHRINK_MODES[mode], _thresholds(levels, thresholds),
                                   _stream(x.device)))
    return y


def shrink2d(x: torch.Tensor, levels: int, thresholds, mode: str = "hard",
             out: torch.Tensor | None = None) -> torch.Tensor:
    """Fused 2D analysis -> thresholding of the level-j bands with
    thresholds[j-1] -> synthesis, on the last two axes."""
    x = _prep(x, 2)
    y = _out(x, out)
    h, w = x.shape[-2], x.shape[-1]
    batch = x.numel() // (h * w) if h * w > 0 else 0
    _abi.check(_abi.haar_shrink_2d(x.data_ptr(), y.data_ptr(), h, w, int(levels), batch, dtype_code(x),
                                   SHRINK_MODES[mode], _thresholds(levels, thresholds),
                                   _stream(x.device)))
    return y


def direct1d(x: torch.Tensor, levels: int, inverse: bool = False, out: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None) -> torch.Tensor:
    """The same transform through the direct (convolve-then-decimate) filter
    bank of Fig. 1 / Fig. 5, one level per pass with the full-rate streams in
    a workspace; for comparison with fwd1d / inv1d."""
    x = _prep(x, 1)
    y = _out(x, out)
    n = x.shape[-1]
    batch = x.numel() // n if n > 0 else 0
    need = _abi.haar_direct_workspace_size(n, batch)
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(max(need, 4), dtype=torch.uint8, device=x.device)
    _abi.check(_abi.haar_direct_1d(x.data_ptr(), y.data_ptr(), n, int(levels), batch, dtype_code(x),
                                   int(inverse), workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(), _stream(x.device)))
    return y


def tune_2d(shape, levels: int, dtype=torch.float32, inverse: bool = False, device="cuda") -> int:
    """Time the 2D tile candidates for [batch, h, w] and record the fastest; returns its index."""
    *lead, h, w = shape
    batch = 1
    for d in lead:
        batch *= d
    esz = torch.tensor([], dtype=dtype).element_size()
    nbytes = 2 * batch * h * w * esz + 64
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
    choice = ctypes.c_int32(-1)
    _abi.check(_abi.haar_tune_2d(DTYPE_CODES[dtype], int(inverse), h, w, int(levels), batch,
                                 scratch.data_ptr(), nbytes, _stream(scratch.device),
                                 ctypes.byref(choice)))
    return choice.value


def tune_1d(shape, levels: int, dtype=torch.float32, inverse: bool = False, device="cuda") -> int:
    """Time the 1D chunk candidates for [batch, n] and record the fastest; returns its index."""
    *lead, n = shape
    batch = 1
    for d in lead:
        batch *= d
    esz = torch.tensor([], dtype=dtype).element_size()
    nbytes = 2 * batch * n * esz + 64
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
    choice = ctypes.c_int32(-1)
    _abi.check(_abi.haar_tune_1d(DTYPE_CODES[dtype], int(inverse), n, int(levels), batch,
                                 scratch.data_ptr(), nbytes, _stream(scratch.device),
                                 ctypes.byref(choice)))
    return choice.value
