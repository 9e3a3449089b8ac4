"""Fused shrinkage (analysis -> threshold the details -> synthesis, one HBM
pass) against the FP64 oracle's shrink, element by element.

Hard thresholding decides keep/zero from a coefficient's magnitude; the GPU
computes the coefficients in FP32, the oracle in FP64.  Thresholds are
therefore placed in gaps of the oracle's coefficient magnitudes, at least
1e-4 * RMS(x) away from every one of them, where both precisions take the
same decision (the FP32 coefficient error is below 1e-5 * RMS(x))."""
import numpy as np
import pytest

import oracle
from gpu_util import check_lowp_signal, check_signal, rms, to_device, to_host
from workloads import generators as G

pytestmark = pytest.mark.gpu

MODES = {0: "hard", 1: "soft"}


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform


def _pick(mags, q, margin):
    """A threshold near the q-quantile of `mags`, in a gap wider than 2 * margin."""
    m = np.unique(np.sort(mags))
    if m.size == 0:
        return 1.0
    k0 = min(int(q * m.size), m.size - 1)
    for k in list(range(k0, m.size - 1)) + list(range(k0 - 1, -1, -1)):
        if m[k + 1] - m[k] > 2 * margin:
            return float(0.5 * (m[k] + m[k + 1]))
    return float(m[-1] + 2 * margin)


def _thresholds_1d(xw, L, q, margin):
    n = xw.shape[-1]
    c = oracle.fwd_1d(xw, L)
    ns = oracle.sizes_1d(n, L)
    return [_pick(np.abs(c[..., ns[j]:ns[j - 1]]).ravel(), q, margin) for j in range(1, L + 1)]


def _thresholds_2d(xw, L, q, margin):
    h, w = xw.shape[-2], xw.shape[-1]
    c = oracle.fwd_2d(xw, L)
    sl = oracle.band_slices_2d(h, w, L)
    out = []
    for j in range(1, L + 1):
        mags = np.concatenate([np.abs(c[(..., *sl[(b, j)])]).ravel() for b in ("HL", "LH", "HH")])
        out.append(_pick(mags, q, margin))
    return out


def _check(got, ref, x_rms, dt, what):
    (check_signal if dt == G.F32 else check_lowp_signal)(got, ref, x_rms, dt, what)


# full 4096-sample chunks at every kind of depth (in-thread only, wavefront,
# across wavefronts), ragged tails, and short signals (one partial chunk)
CASES_1D = [(1, 0), (5, 2), (64, 6), (1000, 3), (4096, 12), (4097, 12), (12345, 5), (65536, 12),
            (3000, 12), (8192, 3), (8192, 8), (16384, 11), (8193, 4)]


@pytest.mark.parametrize("dt", [G.F32, G.BF16, G.F16])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n,L", CASES_1D, ids=lambda v: str(v))
def test_shrink_1d(T, dt, mode, n, L):
    rng = np.random.default_rng(n + 7 * L + 100 * mode + dt)
    xs = G.to_storage(rng.standard_normal((3, n)) * 2.0 + 0.5, dt)
    xw = G.widen(xs, dt)
    r = rms(xw)
    thr = _thresholds_1d(xw, L, 0.6, 1e-4 * r) if L > 0 else []
    ref = oracle.shrink_1d(xw, L, mode, thr) if L > 0 else xw
    got = G.widen(to_host(T.shrink1d(to_device(xs, dt), L, thr, MODES[mode]), dt), dt)
    for b in range(3):
        _check(got[b], ref[b], rms(xw[b]), dt, f"shrink1d n={n} L={L} mode {mode} item {b}")


CASES_2D = [(1, 1, 0), (7, 5, 3), (32, 128, 5), (33, 129, 4), (100, 102, 3), (64, 1090, 5),
            (257, 300, 5), (96, 520, 2), (2, 70, 1)]


@pytest.mark.parametrize("dt", [G.F32, G.BF16, G.F16])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("h,w,L", CASES_2D, ids=lambda v: str(v))
def test_shrink_2d(T, dt, mode, h, w, L):
    rng = np.random.default_rng(h * 1000 + w + 7 * L + 100 * mode + dt)
    xs = G.to_storage(rng.standard_normal((2, h, w)) * 3.0 + 1.0, dt)
    xw = G.widen(xs, dt)
    r = rms(xw)
    thr = _thresholds_2d(xw, L, 0.5, 1e-4 * r) if L > 0 else []
    ref = oracle.shrink_2d(xw, L, mode, thr) if L > 0 else xw
    got = G.widen(to_host(T.shrink2d(to_device(xs, dt), L, thr, MODES[mode]), dt), dt)
    for b in range(2):
        _check(got[b], ref[b], rms(xw[b]), dt, f"shrink2d {h}x{w} L={L} mode {mode} item {b}")


def test_shrink_limits(T):
    """Threshold 0 reconstructs the input; +inf leaves the 2^L block means."""
    import torch
    x = torch.randn(2, 256, 512, device="cuda")
    y0 = T.shrink2d(x, 5, 0.0, "hard")
    assert float((y0 - x).abs().max()) <= 1e-5 * float(x.pow(2).mean().sqrt())
    yi = T.shrink2d(x, 5, float("inf"), "soft")
    means = x.reshape(2, 8, 32, 16, 32).mean(dim=(2, 4))
    want = means.repeat_interleave(32, dim=1).repeat_interleave(32, dim=2)
    assert float((yi - want).abs().max()) <= 1e-5 * float(x.pow(2).mean().sqrt())
    x1 = torch.randn(3, 8192, device="cuda")
    yi1 = T.shrink1d(x1, 12, float("inf"), "hard")
    want1 = x1.reshape(3, 2, 4096).mean(dim=2).repeat_interleave(4096, dim=1)
    assert float((yi1 - want1).abs().max()) <= 1e-5 * float(x1.pow(2).mean().sqrt())


def test_shrink_full_size_image(T):
    """The 4096 x 4096 smooth image, 5 levels, soft thresholds per level."""
    xs = G.config2()
    xw = xs.astype(np.float64)
    thr = [40.0, 20.0, 10.0, 5.0, 2.5]
    ref = oracle.shrink_2d(xw, 5, 1, thr)
    got = to_host(T.shrink2d(to_device(xs, G.F32), 5, thr, "soft"), G.F32).astype(np.float64)
    rel = check_signal(got, ref, rms(xw), G.F32, "shrink2d 4096^2")
    print(f"4096^2 soft shrink err/RMS {rel:.3e}")
