"""3D parity: libhaar's separable volume transform (HIP, through the C ABI)
against the FP64 oracle, element by element.

FP32 gate for 3D coefficients: |gpu - oracle| <= 1e-5 * RMS(x) + ulp(oracle)
per element.  The 3D approximation grows by 2^(3/2) per level, so at depth 6
a positive volume's LLL values exceed 2^8 * RMS(x) and one correct FP32
rounding of them already exceeds 1e-5 * RMS(x); the extra unit in the last
place of the value admits exactly that rounding.  Reconstructions use the
plain 1e-5 * RMS(x) gate; BF16/FP16 use the one-ulp and per-band gates of
the 1D/2D tests."""
import numpy as np
import pytest

import oracle
from gpu_util import (FP32_TOL, check_lowp_coeffs, check_lowp_signal, check_roundtrip, check_signal,
                      rms, to_device, to_host, ulp)
from workloads import generators as G

pytestmark = pytest.mark.gpu

DTYPES = [G.F32, G.BF16, G.F16]
# (d, h, w): one interior tile, several, edges on each axis, odd and tiny
# volumes, lines along each axis, mixes of interior and edge tiles
SHAPES = [(8, 8, 64), (16, 16, 128), (9, 8, 64), (8, 13, 64), (8, 8, 100), (5, 7, 9), (1, 1, 1),
          (1, 1, 130), (3, 1, 5), (17, 19, 67), (32, 24, 192), (24, 16, 320), (1, 40, 72)]


def _levels_for(d, h, w):
    m = int(np.ceil(np.log2(max(d, h, w)))) if max(d, h, w) > 1 else 0
    return [l for l in sorted({1, 2, 3, 4, m}) if 1 <= l <= m] or [0]


def _cases():
    return [(dt, s, L) for dt in DTYPES for s in SHAPES for L in _levels_for(*s)]


def _input(dt, batch, d, h, w, seed):
    rng = np.random.default_rng(seed)
    return G.to_storage(rng.standard_normal((batch, d, h, w)) * 3.0 + 1.0, dt)


def check_coeffs_f32(got, ref, x_rms, what):
    dev = np.abs(got - ref)
    lim = FP32_TOL * x_rms + ulp(ref, G.F32)
    bad = dev > lim
    assert not bad.any(), (f"{what}: {int(bad.sum())} coefficients beyond 1e-5*RMS(x) + ulp, "
                           f"worst {float(dev.max()):.3e} (RMS(x) {x_rms:.3e})")
    return float(dev.max()) / x_rms if x_rms > 0 else 0.0


def _check_fwd(got, ref, xw, dt, L, what):
    d, h, w = ref.shape[-3:]
    for b in range(ref.shape[0]):
        r = rms(xw[b])
        if dt == G.F32:
            check_coeffs_f32(got[b], ref[b], r, f"{what} item {b}")
        else:
            check_lowp_coeffs(got[b], ref[b], r, dt, oracle.band_slices_3d(d, h, w, L), f"{what} item {b}")


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform


@pytest.mark.parametrize("dt,shape,L", _cases(), ids=lambda v: str(v))
def test_fwd_inv_3d(T, dt, shape, L):
    batch = 2
    d, h, w = shape
    xs = _input(dt, batch, d, h, w, seed=d * 10007 + h * 101 + w + 7 * L + dt)
    xw = G.widen(xs, dt)
    ref = oracle.fwd_3d(xw, L)
    y = T.fwd3d(to_device(xs, dt), L)
    _check_fwd(G.widen(to_host(y, dt), dt), ref, xw, dt, L, f"fwd3d {shape} L={L}")
    # synthesis of the stored oracle coefficients
    cs = G.to_storage(ref, dt)
    cw = G.widen(cs, dt)
    xref = oracle.inv_3d(cw, L)
    xr = G.widen(to_host(T.inv3d(to_device(cs, dt), L), dt), dt)
    for b in range(batch):
        chk = check_signal if dt == G.F32 else check_lowp_signal
        chk(xr[b], xref[b], rms(cw[b]), dt, f"inv3d {shape} L={L} item {b}")
    # perfect reconstruction of the GPU's own coefficients
    x2 = G.widen(to_host(T.inv3d(y, L), dt), dt)
    for b in range(batch):
        check_roundtrip(x2[b], xw[b], dt, f"round trip {shape} L={L} item {b}")


# The levels after the first pass run in one tail launch when the region
# left by that pass is small; the last two shapes leave regions too large for
# it (33 x 32 x 32 and 4 x 4 x 2049), so chained passes over scratch run there.
DEEP = [(G.F32, (64, 64, 64), 6), (G.F32, (40, 48, 200), 8), (G.F32, (16, 16, 1024), 10),
        (G.F32, (72, 24, 136), 5), (G.F32, (64, 64, 512), 4), (G.F32, (80, 72, 704), 5),
        (G.BF16, (64, 64, 512), 4), (G.F16, (72, 24, 136), 5), (G.BF16, (64, 64, 1024), 6),
        (G.F32, (264, 256, 256), 7), (G.BF16, (32, 32, 16392), 4)]


@pytest.mark.parametrize("dt,shape,L", DEEP, ids=lambda v: str(v))
def test_deep_3d_phantom(T, dt, shape, L):
    """Depths beyond one fused pass (LLL chained through pair scratch; the
    larger shapes give the later passes interior tiles too) on the CT-like
    phantom, whose positive mean makes the deep LLL values large."""
    xs = G.to_storage(G.phantom_volume(np.random.default_rng(sum(shape) + L), *shape)[None], dt)
    xw = G.widen(xs, dt)
    ref = oracle.fwd_3d(xw, L)
    y = T.fwd3d(to_device(xs, dt), L)
    _check_fwd(G.widen(to_host(y, dt), dt), ref, xw, dt, L, f"deep fwd3d {shape} L={L}")
    cs = G.to_storage(ref, dt)
    xref = oracle.inv_3d(G.widen(cs, dt), L)
    xr = G.widen(to_host(T.inv3d(to_device(cs, dt), L), dt), dt)
    (check_signal if dt == G.F32 else check_lowp_signal)(xr[0], xref[0], rms(xw), dt, f"deep inv3d {shape} L={L}")


@pytest.mark.parametrize("dt", DTYPES)
def test_levels_zero_and_batch_zero_3d(T, dt):
    import torch
    xs = _input(dt, 2, 3, 9, 13, 1)
    y = T.fwd3d(to_device(xs, dt), 0)
    assert np.array_equal(to_host(y, dt), xs)
    x = torch.empty((0, 8, 8, 8), device="cuda")
    assert T.fwd3d(x, 3).shape == (0, 8, 8, 8)


def test_constant_volume_exact(T):
    """Details of a constant are exactly zero; LLL_L = c 2^(3L/2) (2^L | size)
    to one rounding."""
    import torch
    c = 1.75
    x = torch.full((2, 16, 32, 128), c, device="cuda")
    for L in (1, 2, 3, 4):
        y = T.fwd3d(x, L).cpu().numpy().astype(np.float64)
        dL, hL, wL = 16 >> L, 32 >> L, 128 >> L
        want = np.float32(c * 2.0 ** (1.5 * L))
        assert np.all(np.abs(y[:, :dL, :hL, :wL] - want) <= ulp(np.array([want]), G.F32)[0])
        m = np.ones((16, 32, 128), bool)
        m[:dL, :hL, :wL] = False
        assert np.all(y[:, m] == 0.0)


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
def test_full_size_phantom_volumes(T, dt):
    """The suite's workload size: 4 x 256^3 phantom volumes, 3 levels (one
    fused pass), every coefficient against the oracle; then L8 (three
    passes) on one volume."""
    import torch
    rng = np.random.default_rng(8)
    base = G.phantom_volume(rng, 256, 256, 256)
    x64 = np.stack([base + rng.normal(0.0, 0.02, base.shape) for _ in range(4)])
    xs = G.to_storage(x64, dt)
    del x64
    xw = G.widen(xs, dt)
    ref = oracle.fwd_3d(xw, 3)
    y = T.fwd3d(to_device(xs, dt), 3)
    _check_fwd(G.widen(to_host(y, dt), dt), ref, xw, dt, 3, f"fwd3d 4x256^3 {G.DTYPE_NAMES[dt]}")
    x2 = G.widen(to_host(T.inv3d(y, 3), dt), dt)
    for b in range(4):
        check_roundtrip(x2[b], xw[b], dt, f"round trip 4x256^3 item {b}")
    del y, ref, x2
    torch.cuda.empty_cache()
    ref8 = oracle.fwd_3d(xw[:1], 8)
    y8 = T.fwd3d(to_device(xs[:1], dt), 8)
    _check_fwd(G.widen(to_host(y8, dt), dt), ref8, xw[:1], dt, 8, f"fwd3d 256^3 L8 {G.DTYPE_NAMES[dt]}")


def test_autograd_3d_adjoint(T):
    """Backward of the 3D analysis is the oracle's transpose W^T g (the
    synthesis), and backward of the synthesis is the analysis: checked on an
    odd volume through torch.autograd with the oracle's adjoint."""
    import torch
    from paper_1002_2184_amd import autograd as AG
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 9, 20, 70))
    g = rng.standard_normal((2, 9, 20, 70))
    L = 4
    xt = torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    (gx,) = torch.autograd.grad(AG.HaarFwd3D.apply(xt, L), xt, gt)
    want = oracle.inv_3d(g.astype(np.float32).astype(np.float64), L)
    check_signal(gx.cpu().numpy().astype(np.float64), want, rms(g), G.F32, "HaarFwd3D backward")
    (gy,) = torch.autograd.grad(AG.HaarInv3D.apply(xt, L), xt, gt)
    want = oracle.fwd_3d(g.astype(np.float32).astype(np.float64), L)
    check_coeffs_f32(gy.cpu().numpy().astype(np.float64), want, rms(g), "HaarInv3D backward")
