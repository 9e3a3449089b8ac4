"""The direct (convolve-then-decimate) filter bank on the GPU against the
oracle's direct bank and its fast bank (the two must agree), element by
element."""
import numpy as np
import pytest

import oracle
from gpu_util import band_views, check_lowp_coeffs, check_lowp_signal, check_signal, rms, to_device, to_host
from workloads import generators as G

pytestmark = pytest.mark.gpu

CASES = [(1, 0), (2, 1), (7, 3), (64, 6), (1000, 5), (4097, 12), (12345, 10), (65536, 16)]


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
@pytest.mark.parametrize("n,L", CASES, ids=lambda v: str(v))
def test_direct_1d(T, dt, n, L):
    rng = np.random.default_rng(7 * n + L + dt)
    xs = G.to_storage(rng.standard_normal((2, n)) * 2.0 + 0.5, dt)
    xw = G.widen(xs, dt)
    ref = oracle.direct_fwd_1d(xw, L)
    np.testing.assert_allclose(ref, oracle.fwd_1d(xw, L), rtol=0, atol=1e-12 * max(1.0, rms(xw)))
    y = G.widen(to_host(T.direct1d(to_device(xs, dt), L), dt), dt)
    cs = G.to_storage(ref, dt)
    xr = G.widen(to_host(T.direct1d(to_device(cs, dt), L, inverse=True), dt), dt)
    xref = oracle.direct_inv_1d(G.widen(cs, dt), L)
    for b in range(2):
        what = f"direct n={n} L={L} item {b}"
        if dt == G.F32:
            check_signal(y[b], ref[b], rms(xw[b]), dt, what + " fwd")
            check_signal(xr[b], xref[b], rms(xw[b]), dt, what + " inv")
        else:
            check_lowp_coeffs(y[b], ref[b], rms(xw[b]), dt, band_views(n, L), what + " fwd")
            check_lowp_signal(xr[b], xref[b], rms(xw[b]), dt, what + " inv")


def test_direct_equals_fast_on_gpu(T):
    """The two banks on the GPU give the same coefficients (FP32 rounding apart)."""
    import torch
    x = torch.randn(4, 50000, device="cuda")
    a = T.fwd1d(x, 14)
    b = T.direct1d(x, 14)
    scale = float(x.pow(2).mean().sqrt())
    assert float((a - b).abs().max()) <= 1e-5 * scale
    assert float((T.direct1d(b, 14, inverse=True) - x).abs().max()) <= 1e-5 * scale
