"""2D parity: libhaar (HIP, through the C ABI) against the FP64 oracle, element by element."""
import numpy as np
import pytest

import oracle
from gpu_util import (band_views, check_lowp_coeffs, check_lowp_signal, check_roundtrip,
                      check_signal, rms, to_device, to_host)
from workloads import generators as G

pytestmark = pytest.mark.gpu

DTYPES = [G.F32, G.BF16, G.F16]
# (h, w): degenerate, single tile, multi-tile full, ragged, unaligned rows; full
# tiles whose rows and band origins start at odd elements (W/2 or W/4 odd);
# wide rows of whole cache lines in every dtype (nontemporal loads, and paced
# stores for 16-bit data)
SHAPES = [(1, 1), (1, 9), (7, 1), (2, 2), (3, 5), (32, 32), (32, 128), (64, 256), (33, 129),
          (100, 102), (130, 70), (257, 300), (96, 520), (64, 1090), (96, 1546), (64, 1025),
          (160, 578), (64, 2048)]


def _levels_for(h, w):
    m = int(np.ceil(np.log2(max(h, w)))) if max(h, w) > 1 else 0
    lv = sorted({min(1, m), min(2, m), min(3, m), min(5, m), m})
    return [l for l in lv if l >= 1] or [0]


def _cases():
    out = []
    for dt in DTYPES:
        for (h, w) in SHAPES:
            for L in _levels_for(h, w):
                out.append((dt, h, w, L))
    return out


def _input(dt, batch, h, w, seed):
    rng = np.random.default_rng(seed)
    x64 = rng.standard_normal((batch, h, w)) * 3.0 + 1.0
    return G.to_storage(x64, dt)


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform


@pytest.mark.parametrize("dt,h,w,L", _cases(), ids=lambda v: str(v))
def test_fwd_inv_2d(T, dt, h, w, L):
    batch = 3
    xs = _input(dt, batch, h, w, seed=h * 1000 + w + 7 * L + dt)
    xw = G.widen(xs, dt)
    ref = oracle.fwd_2d(xw, L)
    y = T.fwd2d(to_device(xs, dt), L)
    yw = G.widen(to_host(y, dt), dt)
    for b in range(batch):
        r = rms(xw[b])
        if dt == G.F32:
            check_signal(yw[b], ref[b], r, dt, f"fwd {h}x{w} L={L} item {b}")
        else:
            check_lowp_coeffs(yw[b], ref[b], r, dt, band_views((h, w), L), f"fwd {h}x{w} L={L} item {b}")
    # inverse of the (stored) oracle coefficients
    cs = G.to_storage(ref, dt)
    cw = G.widen(cs, dt)
    xref = oracle.inv_2d(cw, L)
    xr = G.widen(to_host(T.inv2d(to_device(cs, dt), L), dt), dt)
    for b in range(batch):
        chk = check_signal if dt == G.F32 else check_lowp_signal
        chk(xr[b], xref[b], rms(cw[b]), dt, f"inv {h}x{w} L={L} item {b}")
    # perfect reconstruction of the GPU's own coefficients
    x2 = G.widen(to_host(T.inv2d(y, L), dt), dt)
    for b in range(batch):
        check_roundtrip(x2[b], xw[b], dt, f"round trip {h}x{w} L={L} item {b}")


@pytest.mark.parametrize("dt", DTYPES)
def test_levels_zero_copies(T, dt):
    xs = _input(dt, 2, 9, 13, 1)
    y = T.fwd2d(to_device(xs, dt), 0)
    assert np.array_equal(to_host(y, dt), xs)


def test_batch_zero(T):
    import torch
    x = torch.empty((0, 8, 8), device="cuda")
    assert T.fwd2d(x, 3).shape == (0, 8, 8)


def test_constant_image_exact(T):
    """Details of a constant are exactly zero; LL_L = c 2^L exactly (2^L | size)."""
    import torch
    c = 3.25
    x = torch.full((2, 64, 96), c, device="cuda")
    for L in (1, 3, 5):
        y = T.fwd2d(x, L).cpu().numpy()
        hL, wL = 64 >> L, 96 >> L
        assert np.all(y[:, :hL, :wL] == c * 2.0 ** L)
        m = np.ones((64, 96), bool)
        m[:hL, :wL] = False
        assert np.all(y[:, m] == 0.0)


def test_deep_levels_multi_pass(T):
    """Levels beyond one fused pass (intermediate approximations in scratch)."""
    dt = G.F32
    for (h, w, L) in [(256, 256, 8), (300, 170, 9), (64, 1024, 10)]:
        xs = _input(dt, 2, h, w, seed=h + w)
        xw = G.widen(xs, dt)
        ref = oracle.fwd_2d(xw, L)
        y = T.fwd2d(to_device(xs, dt), L)
        yw = G.widen(to_host(y, dt), dt)
        for b in range(2):
            check_signal(yw[b], ref[b], rms(xw[b]), dt, f"deep fwd {h}x{w} L={L}")
        xr = G.widen(to_host(T.inv2d(to_device(G.to_storage(ref, dt), dt), L), dt), dt)
        xref = oracle.inv_2d(G.widen(G.to_storage(ref, dt), dt), L)
        for b in range(2):
            check_signal(xr[b], xref[b], rms(xw[b]), dt, f"deep inv {h}x{w} L={L}")


def test_offset_views_unaligned(T):
    """Inputs/outputs at odd element offsets take the scalar path and still match."""
    import torch
    h, w, L = 40, 72, 3
    base = torch.randn(h * w + 1, device="cuda")
    x = base[1:].view(h, w)                       # 4-byte aligned only
    outbuf = torch.empty(h * w + 1, device="cuda")
    y = T.fwd2d(x, L, out=outbuf[1:].view(h, w))
    ref = oracle.fwd_2d(x.cpu().numpy().astype(np.float64), L)
    check_signal(y.cpu().numpy().astype(np.float64), ref, rms(ref), G.F32, "offset fwd")


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
def test_tile_configs_agree(T, dt):
    """Every tile shape (and thread map) gives the oracle's result at every
    depth of one pass, on shapes with interior and edge tiles."""
    from paper_1002_2184_amd import _abi
    cases = []
    for shape in ((2, 200, 330), (1, 256, 1024)):
        xs = _input(dt, *shape, 5)
        xw = G.widen(xs, dt)
        for L in (1, 2, 3, 4, 5):
            ref = oracle.fwd_2d(xw, L)
            cs = G.to_storage(ref, dt)
            cases.append((shape, L, xs, xw, ref, cs, oracle.inv_2d(G.widen(cs, dt), L)))
    try:
        for c in range(_abi.haar_tune_candidates_2d(dt)):
            assert _abi.haar_force_config_2d(dt, c) == 0
            for shape, L, xs, xw, ref, cs, xref in cases:
                y = G.widen(to_host(T.fwd2d(to_device(xs, dt), L), dt), dt)
                xr = G.widen(to_host(T.inv2d(to_device(cs, dt), L), dt), dt)
                for b in range(shape[0]):
                    what = f"config {c} {shape} L={L} item {b}"
                    if dt == G.F32:
                        check_signal(y[b], ref[b], rms(xw[b]), dt, what)
                        check_signal(xr[b], xref[b], rms(xw[b]), dt, what + " inv")
                    else:
                        check_lowp_coeffs(y[b], ref[b], rms(xw[b]), dt, band_views(shape[1:], L), what)
                        check_lowp_signal(xr[b], xref[b], rms(xw[b]), dt, what + " inv")
    finally:
        _abi.haar_force_config_2d(dt, -1)


def test_config2_full_size():
    """The 4096 x 4096 smooth FP32 image, 5 levels: every coefficient and sample."""
    from paper_1002_2184_amd import transform as T
    xs = G.config2()
    xw = xs.astype(np.float64)
    ref = oracle.fwd_2d(xw, 5)
    y = T.fwd2d(to_device(xs, G.F32), 5)
    yw = to_host(y, G.F32).astype(np.float64)
    rel = check_signal(yw, ref, rms(xw), G.F32, "config2 fwd")
    xr = to_host(T.inv2d(y, 5), G.F32).astype(np.float64)
    rel2 = check_signal(xr, xw, rms(xw), G.F32, "config2 round trip")
    xr2 = to_host(T.inv2d(to_device(ref.astype(np.float32), G.F32), 5), G.F32).astype(np.float64)
    xref = oracle.inv_2d(ref.astype(np.float32).astype(np.float64), 5)
    rel3 = check_signal(xr2, xref, rms(xw), G.F32, "config2 inv")
    print(f"config2 err/RMS: fwd {rel:.3e}  roundtrip {rel2:.3e}  inv {rel3:.3e}")
