"""Helpers of the GPU parity tests: device transfer of storage arrays and the gates.

Gates (FP64 oracle as reference, input = the exact stored values widened):
* FP32 storage: max |gpu - oracle| <= 1e-5 * RMS(x) per item (x = the signal
  domain input, whose RMS equals the coefficients' RMS by Parseval).
* BF16 / FP16 storage, signal-domain outputs (synthesis of stored
  coefficients): every value within one unit in the last place of the
  correctly rounded oracle value (plus an absolute floor of 1e-6 * RMS(x)).
  The max-abs gate 1e-2 * RMS(x) is checked on the U[0, 1] images of the
  batched BF16 workload (test_gpu_precision); for data whose peak exceeds
  ~2.5 RMS a single BF16 rounding of the peak already exceeds it.
* BF16 / FP16 round trip inv(fwd(x)) (two storage roundings): RMS error
  <= 1e-2 * RMS(x).
* BF16 / FP16 storage, coefficients (analysis): every value within one unit
  in the last place of the correctly rounded oracle value (plus an absolute
  floor of 1e-6 * RMS(x) for values that cancel to ~0), and per band
  (level j, subband) max |err| <= 1e-2 * max |oracle band| (band_gate=True).
  Relative to the band RMS the same limit cannot hold for bands whose peak
  exceeds ~2.5 RMS (one correct BF16 rounding of the peak already exceeds
  it); the per-band RMS error relative to the band RMS is returned for the
  report.
"""
from __future__ import annotations

import numpy as np

import oracle
from workloads import generators as G

FP32_TOL = 1e-5
LOWP_TOL = 1e-2


def torch_dtype(dt):
    import torch
    return {G.F32: torch.float32, G.BF16: torch.bfloat16, G.F16: torch.float16}[dt]


def to_device(stored, dt):
    import torch
    a = np.ascontiguousarray(stored)
    if dt == G.F32:
        return torch.from_numpy(a).cuda()
    return torch.from_numpy(a.view(np.int16)).cuda().view(torch_dtype(dt))


def to_host(t, dt):
    import torch
    if dt == G.F32:
        return t.detach().cpu().numpy()
    return t.detach().view(torch.int16).cpu().numpy().view(np.uint16)


def rms(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.mean(a * a))) if a.size else 0.0


def ulp(v, dt):
    """Unit in the last place of storage-format values v (float64 array)."""
    av = np.abs(np.asarray(v, dtype=np.float64))
    if dt == G.BF16:
        mant, emin = 7, -126
    elif dt == G.F16:
        mant, emin = 10, -14
    else:
        mant, emin = 23, -126
    e = np.floor(np.log2(np.where(av > 0, av, 2.0 ** emin)))
    e = np.maximum(e, emin)
    return 2.0 ** (e - mant)


def err_report(gpu64, ref64, scale):
    err = float(np.max(np.abs(gpu64 - ref64))) if gpu64.size else 0.0
    return err, (err / scale if scale > 0 else err)


def check_signal(gpu64, ref64, x_rms, dt, what=""):
    """Signal-domain (or FP32 coefficient) gate: max err <= tol * RMS(x)."""
    tol = FP32_TOL if dt == G.F32 else LOWP_TOL
    err, rel = err_report(gpu64, ref64, x_rms)
    assert rel <= tol, f"{what}: max err {err:.3e} = {rel:.3e} * RMS(x) > {tol:g}"
    return rel


def check_lowp_signal(gpu64, ref64, x_rms, dt, what=""):
    """Reduced-precision signal outputs: within one ulp of RNE(oracle)."""
    rounded = G.widen(G.to_storage(ref64, dt), dt)
    dev = np.abs(gpu64 - rounded)
    bad = dev > ulp(rounded, dt) + 1e-6 * x_rms
    assert not bad.any(), (f"{what}: {int(bad.sum())} values more than 1 ulp from RNE(oracle), "
                           f"worst {float(dev.max()):.3e}")
    return err_report(gpu64, ref64, x_rms)[1]


def check_roundtrip(gpu64, x64, dt, what=""):
    """inv(fwd(x)) vs x: max err (FP32) or RMS err (reduced precision) over RMS(x)."""
    r = rms(x64)
    if dt == G.F32:
        return check_signal(gpu64, x64, r, dt, what)
    rel = rms(gpu64 - x64) / r
    assert rel <= LOWP_TOL, f"{what}: RMS err {rel:.3e} * RMS(x) > {LOWP_TOL:g}"
    return rel


def band_views(shape2d_or_n, levels):
    if isinstance(shape2d_or_n, tuple):
        return oracle.band_slices_2d(shape2d_or_n[0], shape2d_or_n[1], levels)
    return oracle.band_slices_1d(shape2d_or_n, levels)


def check_lowp_coeffs(gpu64, ref64, x_rms, dt, bands, what="", band_gate=False):
    """One-ulp check (and optionally the per-band gate) for reduced-precision
    coefficients; returns the worst per-band max err / RMS(band).

    gpu64/ref64: one item's coefficients (1D vector or 2D array)."""
    rounded = G.widen(G.to_storage(ref64, dt), dt)        # RNE(oracle)
    floor = 1e-6 * x_rms
    dev = np.abs(gpu64 - rounded)
    bad = dev > ulp(rounded, dt) + floor
    assert not bad.any(), (f"{what}: {int(bad.sum())} values more than 1 ulp from RNE(oracle), "
                           f"worst {float(dev.max()):.3e}")
    table = {}
    for key, sl in bands.items():
        g, r = gpu64[sl], ref64[sl]
        if g.size == 0:
            continue
        br = rms(r)
        peak = float(np.max(np.abs(r)))
        err = float(np.max(np.abs(g - r)))
        if band_gate:
            lim = LOWP_TOL * max(peak, floor)
            assert err <= lim, f"{what} band {key}: max err {err:.3e} > 1e-2 * max|band| = {lim:.3e}"
        # the floor: the same measures for the correctly rounded oracle itself
        fl = float(np.max(np.abs(rounded[sl] - r)))
        table[key] = {"max_err_over_band_peak": err / max(peak, floor),
                      "rms_err_over_band_rms": rms(g - r) / max(br, floor),
                      "max_err_over_band_rms": err / max(br, floor),
                      "floor_max_err_over_band_peak": fl / max(peak, floor),
                      "floor_max_err_over_band_rms": fl / max(br, floor)}
    return table
