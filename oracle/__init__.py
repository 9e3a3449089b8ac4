"""FP64 oracle of the fast Haar wavelet transform -- TEST INFRASTRUCTURE ONLY.

The arithmetic lives in ``haar_oracle.c`` (plain C, double precision, built
with gcc into ``liboracle.so`` beside it).  This module only marshals numpy
arrays into it.  It may be imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the library package: the
two share no code.

Functions (all float64 in, float64 out, out-of-place, same shape):

* ``fwd_1d(x, levels)`` / ``inv_1d(y, levels)`` -- fast analysis / synthesis
  banks (Sec. III Eq. (11)-(12) and Fig. 4; Sec. IV Eq. (19) and Fig. 7),
  recursed on the approximation; x has shape ``[..., n]``.
* ``direct_fwd_1d`` / ``direct_inv_1d`` -- the same transform through the
  direct full-rate filter bank of Fig. 1/2 and Eq. (13) (convolve, then
  decimate; up-sample, then convolve).
* ``fwd_2d(x, levels)`` / ``inv_2d(y, levels)`` -- separable 2D on
  ``[..., h, w]``: rows then columns per level, recursion on LL.
* ``fwd_3d(x, levels)`` / ``inv_3d(y, levels)`` -- separable 3D on
  ``[..., d, h, w]``: x, then y, then z per level, recursion on LLL.
* ``l1_grad_2d(x, levels)`` -- loss sum |details| + 0.5 ||LL_L||^2 of the
  2D analysis and its gradient with respect to x (synthesis of the
  coefficient gradient).
* ``filter_taps()`` -- the taps (b0, b1, a0, a1) of Eq. (8), (9), (17), (18).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "haar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle C source with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_levels(levels: int) -> None:
    if not (0 <= int(levels) <= 62):
        raise ValueError(f"levels must be in [0, 62], got {levels}")


class Oracle:
    """ctypes view of one compiled copy of the oracle (normally ``liboracle.so``)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(ctypes.c_double)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        for name in ("oracle_fwd_1d", "oracle_inv_1d", "oracle_direct_fwd_1d",
                     "oracle_direct_inv_1d"):
            fn = getattr(lib, name)
            fn.argtypes = [P, P, i64, i32, i64]
            fn.restype = None
        for name in ("oracle_fwd_2d", "oracle_inv_2d"):
            fn = getattr(lib, name)
            fn.argtypes = [P, P, i64, i64, i32, i64]
            fn.restype = None
        for name in ("oracle_fwd_3d", "oracle_inv_3d"):
            fn = getattr(lib, name)
            fn.argtypes = [P, P, i64, i64, i64, i32, i64]
            fn.restype = None
        lib.oracle_l1_grad_2d.argtypes = [P, P, P, i64, i64, i32, i64]
        lib.oracle_l1_grad_2d.restype = None
        lib.oracle_shrink_1d.argtypes = [P, P, i64, i32, i64, i32, P]
        lib.oracle_shrink_1d.restype = None
        lib.oracle_shrink_2d.argtypes = [P, P, i64, i64, i32, i64, i32, P]
        lib.oracle_shrink_2d.restype = None
        lib.oracle_filter_taps.argtypes = [P, P, P, P]
        lib.oracle_filter_taps.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def _call_1d(self, name, x, levels):
        _check_levels(levels)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim < 1 or x.shape[-1] < 1:
            raise ValueError("1D oracle needs a non-empty last axis")
        n = x.shape[-1]
        y = np.empty_like(x)
        getattr(self.lib, name)(_ptr(x), _ptr(y), n, int(levels), x.size // n)
        return y

    def _call_2d(self, name, x, levels):
        _check_levels(levels)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim < 2 or x.shape[-1] < 1 or x.shape[-2] < 1:
            raise ValueError("2D oracle needs non-empty last two axes")
        h, w = x.shape[-2], x.shape[-1]
        y = np.empty_like(x)
        getattr(self.lib, name)(_ptr(x), _ptr(y), h, w, int(levels), x.size // (h * w))
        return y

    def fwd_1d(self, x, levels):
        """Multi-level fast analysis bank along the last axis (Fig. 4, recursed)."""
        return self._call_1d("oracle_fwd_1d", x, levels)

    def inv_1d(self, y, levels):
        """Multi-level fast synthesis bank along the last axis (Fig. 7, recursed)."""
        return self._call_1d("oracle_inv_1d", y, levels)

    def direct_fwd_1d(self, x, levels):
        """Same transform through the direct convolve-then-decimate bank (Fig. 2)."""
        return self._call_1d("oracle_direct_fwd_1d", x, levels)

    def direct_inv_1d(self, y, levels):
        """Same inverse through the direct up-sample-then-convolve bank (Eq. (13))."""
        return self._call_1d("oracle_direct_inv_1d", y, levels)

    def fwd_2d(self, x, levels):
        """Separable multi-level 2D analysis on the last two axes."""
        return self._call_2d("oracle_fwd_2d", x, levels)

    def inv_2d(self, y, levels):
        """Separable multi-level 2D synthesis on the last two axes."""
        return self._call_2d("oracle_inv_2d", y, levels)

    def _call_3d(self, name, x, levels):
        _check_levels(levels)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim < 3 or min(x.shape[-3:]) < 1:
            raise ValueError("3D oracle needs non-empty last three axes")
        d, h, w = x.shape[-3], x.shape[-2], x.shape[-1]
        y = np.empty_like(x)
        getattr(self.lib, name)(_ptr(x), _ptr(y), d, h, w, int(levels), x.size // (d * h * w))
        return y

    def fwd_3d(self, x, levels):
        """Separable multi-level 3D analysis on the last three axes (x, y, z per level)."""
        return self._call_3d("oracle_fwd_3d", x, levels)

    def inv_3d(self, y, levels):
        """Separable multi-level 3D synthesis (z, y, x per level, levels L..1)."""
        return self._call_3d("oracle_inv_3d", y, levels)

    def l1_grad_2d(self, x, levels):
        """(loss per item, grad_x) of loss = sum |details| + 0.5 * ||LL_L||^2
        of the 2D analysis of x; grad_x = synthesis of (sign(details), LL_L)."""
        _check_levels(levels)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim < 2 or min(x.shape[-2:]) < 1:
            raise ValueError("2D oracle needs non-empty last two axes")
        h, w = x.shape[-2], x.shape[-1]
        g = np.empty_like(x)
        batch = x.size // (h * w)
        loss = np.empty(batch, dtype=np.float64)
        self.lib.oracle_l1_grad_2d(_ptr(x), _ptr(g), _ptr(loss), h, w, int(levels), batch)
        return loss.reshape(x.shape[:-2]), g

    def _thresholds(self, levels, thresholds):
        t = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float64).reshape(-1))
        if t.size != int(levels):
            raise ValueError(f"need one threshold per level ({levels}), got {t.size}")
        return t

    def shrink_1d(self, x, levels, mode, thresholds):
        """Analysis, thresholding of every level-j detail with thresholds[j-1]
        (mode 0 hard, 1 soft), synthesis; along the last axis."""
        _check_levels(levels)
        t = self._thresholds(levels, thresholds)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        n = x.shape[-1]
        y = np.empty_like(x)
        self.lib.oracle_shrink_1d(_ptr(x), _ptr(y), n, int(levels), x.size // n, int(mode), _ptr(t))
        return y

    def shrink_2d(self, x, levels, mode, thresholds):
        """2D analysis, thresholding of the level-j bands with thresholds[j-1]
        (mode 0 hard, 1 soft), synthesis; on the last two axes."""
        _check_levels(levels)
        t = self._thresholds(levels, thresholds)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        h, w = x.shape[-2], x.shape[-1]
        y = np.empty_like(x)
        self.lib.oracle_shrink_2d(_ptr(x), _ptr(y), h, w, int(levels), x.size // (h * w), int(mode),
                                  _ptr(t))
        return y

    def filter_taps(self):
        """(b0, b1, a0, a1), each a length-2 causal FIR tap array."""
        arrs = [np.zeros(2) for _ in range(4)]
        self.lib.oracle_filter_taps(*[_ptr(a) for a in arrs])
        return tuple(arrs)

    def num_threads(self):
        """OpenMP threads the oracle uses."""
        return int(self.lib.oracle_num_threads())


_default = None


def default() -> Oracle:
    """The oracle built from ``haar_oracle.c`` (compiled on first use if missing)."""
    global _default
    if _default is None:
        build()
        _default = Oracle(_LIB)
    return _default


def fwd_1d(x, levels: int) -> np.ndarray:
    return default().fwd_1d(x, levels)


def inv_1d(y, levels: int) -> np.ndarray:
    return default().inv_1d(y, levels)


def direct_fwd_1d(x, levels: int) -> np.ndarray:
    return default().direct_fwd_1d(x, levels)


def direct_inv_1d(y, levels: int) -> np.ndarray:
    return default().direct_inv_1d(y, levels)


def fwd_2d(x, levels: int) -> np.ndarray:
    return default().fwd_2d(x, levels)


def inv_2d(y, levels: int) -> np.ndarray:
    return default().inv_2d(y, levels)


def fwd_3d(x, levels: int) -> np.ndarray:
    return default().fwd_3d(x, levels)


def inv_3d(y, levels: int) -> np.ndarray:
    return default().inv_3d(y, levels)


def band_slices_3d(d: int, h: int, w: int, levels: int):
    """3D packed layout: {'LLL': (z, y, x slices), (code, j): ...} where code
    is a 3-letter string of L/H for the (x, y, z) filters, e.g. 'HLL' = high
    along x only."""
    ds, hs, ws = sizes_1d(d, levels), sizes_1d(h, levels), sizes_1d(w, levels)
    sl = {"LLL": (slice(0, ds[levels]), slice(0, hs[levels]), slice(0, ws[levels]))}
    for j in range(1, levels + 1):
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    if bx == by == bz == 0:
                        continue
                    zs = slice(ds[j], ds[j - 1]) if bz else slice(0, ds[j])
                    ys = slice(hs[j], hs[j - 1]) if by else slice(0, hs[j])
                    xs = slice(ws[j], ws[j - 1]) if bx else slice(0, ws[j])
                    code = ("H" if bx else "L") + ("H" if by else "L") + ("H" if bz else "L")
                    sl[(code, j)] = (zs, ys, xs)
    return sl


def l1_grad_2d(x, levels: int):
    return default().l1_grad_2d(x, levels)


def shrink_1d(x, levels: int, mode: int, thresholds) -> np.ndarray:
    return default().shrink_1d(x, levels, mode, thresholds)


def shrink_2d(x, levels: int, mode: int, thresholds) -> np.ndarray:
    return default().shrink_2d(x, levels, mode, thresholds)


def filter_taps():
    return default().filter_taps()


def num_threads() -> int:
    return default().num_threads()


def sizes_1d(n: int, levels: int):
    """Lengths n_0 = n, n_j = ceil(n_{j-1} / 2) of the approximation at each level."""
    out = [int(n)]
    for _ in range(levels):
        out.append((out[-1] + 1) // 2)
    return out


def band_slices_1d(n: int, levels: int):
    """Slices of the packed layout: {'a': a_L, ('d', j): d_j} (j = 1..levels)."""
    ns = sizes_1d(n, levels)
    sl = {"a": slice(0, ns[levels])}
    for j in range(1, levels + 1):
        sl[("d", j)] = slice(ns[j], ns[j - 1])
    return sl


def band_slices_2d(h: int, w: int, levels: int):
    """2D packed layout: {'LL': (rows, cols), ('HL', j), ('LH', j), ('HH', j)}."""
    hs, ws = sizes_1d(h, levels), sizes_1d(w, levels)
    sl = {"LL": (slice(0, hs[levels]), slice(0, ws[levels]))}
    for j in range(1, levels + 1):
        h0, w0, h1, w1 = hs[j - 1], ws[j - 1], hs[j], ws[j]
        sl[("HL", j)] = (slice(0, h1), slice(w1, w0))
        sl[("LH", j)] = (slice(h1, h0), slice(0, w1))
        sl[("HH", j)] = (slice(h1, h0), slice(w1, w0))
    return sl
