"""1D parity: libhaar (HIP, through the C ABI) against the FP64 oracle, element by element."""
import numpy as np
import pytest

import oracle
from gpu_util import (band_views, check_lowp_coeffs, check_lowp_signal, check_roundtrip,
                      check_signal, rms, to_device, to_host)
from workloads import generators as G

pytestmark = pytest.mark.gpu

DTYPES = [G.F32, G.BF16, G.F16]
# degenerate, one chunk, chunk boundaries, ragged tails, several passes
LENGTHS = [1, 2, 3, 5, 16, 17, 63, 64, 1000, 1024, 2048, 4095, 4096, 4097, 12345, 16384, 65536,
           100003]


def _levels_for(n):
    m = int(np.ceil(np.log2(n))) if n > 1 else 0
    lv = {1, 3, 4, 5, 10, 11, 12, 13, m}
    return sorted(l for l in lv if 1 <= l <= m) or [0]


def _cases():
    return [(dt, n, L) for dt in DTYPES for n in LENGTHS for L in _levels_for(n)]


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform


def _check_fwd_inv(T, dt, n, L, batch=2, seed=0, what=""):
    """Analysis of a seeded signal batch, synthesis of the oracle's stored
    coefficients and the round trip, each against the oracle."""
    rng = np.random.default_rng(seed)
    xs = G.to_storage(rng.standard_normal((batch, n)) * 2.0 + 0.5, dt)
    xw = G.widen(xs, dt)
    ref = oracle.fwd_1d(xw, L)
    y = T.fwd1d(to_device(xs, dt), L)
    yw = G.widen(to_host(y, dt), dt)
    for b in range(batch):
        r = rms(xw[b])
        if dt == G.F32:
            check_signal(yw[b], ref[b], r, dt, f"{what} fwd n={n} L={L} item {b}")
        else:
            check_lowp_coeffs(yw[b], ref[b], r, dt, band_views(n, L), f"{what} fwd n={n} L={L} item {b}")
    cs = G.to_storage(ref, dt)
    cw = G.widen(cs, dt)
    xref = oracle.inv_1d(cw, L)
    xr = G.widen(to_host(T.inv1d(to_device(cs, dt), L), dt), dt)
    for b in range(batch):
        chk = check_signal if dt == G.F32 else check_lowp_signal
        chk(xr[b], xref[b], rms(cw[b]), dt, f"{what} inv n={n} L={L} item {b}")
    x2 = G.widen(to_host(T.inv1d(y, L), dt), dt)
    for b in range(batch):
        check_roundtrip(x2[b], xw[b], dt, f"{what} round trip n={n} L={L} item {b}")


@pytest.mark.parametrize("dt,n,L", _cases(), ids=lambda v: str(v))
def test_fwd_inv_1d(T, dt, n, L):
    _check_fwd_inv(T, dt, n, L, seed=n * 31 + L + dt)


def test_constant_signal_exact(T):
    import torch
    c = -1.75
    x = torch.full((3, 8192), c, device="cuda")
    for L in (1, 4, 10, 12, 13):
        y = T.fwd1d(x, L).cpu().numpy()
        nL = 8192 >> L
        np.testing.assert_allclose(y[:, :nL], c * 2.0 ** (L / 2), rtol=2e-7)
        if L % 2 == 0:
            assert np.all(y[:, :nL] == c * 2.0 ** (L / 2))
        assert np.all(y[:, nL:] == 0.0)


def test_config1_full_size(T):
    """One N(0,1) FP32 signal of 65536 samples, 16 levels, every coefficient."""
    xs = G.config1()
    xw = xs.astype(np.float64)
    ref = oracle.fwd_1d(xw, 16)
    y = T.fwd1d(to_device(xs, G.F32), 16)
    rel = check_signal(to_host(y, G.F32).astype(np.float64), ref, rms(xw), G.F32, "config1 fwd")
    xr = to_host(T.inv1d(y, 16), G.F32).astype(np.float64)
    rel2 = check_signal(xr, xw, rms(xw), G.F32, "config1 round trip")
    print(f"config1 err/RMS: fwd {rel:.3e} round trip {rel2:.3e}")


def test_config3_signals_sample(T):
    """Sine-mix signals of lengths 2^10..2^20 at full depth (a sample of the batch)."""
    sigs = G.config3(count=12)
    for s in sigs:
        n = s.shape[0]
        L = int(np.log2(n))
        xw = s.astype(np.float64)
        ref = oracle.fwd_1d(xw, L)
        y = T.fwd1d(to_device(s, G.F32), L)
        check_signal(to_host(y, G.F32).astype(np.float64), ref, rms(xw), G.F32, f"config3 n={n}")
        xr = to_host(T.inv1d(y, L), G.F32).astype(np.float64)
        check_signal(xr, xw, rms(xw), G.F32, f"config3 round trip n={n}")


# Chunk shapes a tuning table or haar_tune_1d can select (threads x samples
# per thread): 0: 256 x 16 (default), 1: 1024 x 16, 2: 64 x 16, 3: 128 x 16,
# 4: 256 x 16 without the XCD-contiguous chunk order.
CHUNKS = {0: 4096, 1: 16384, 2: 1024, 3: 2048, 4: 4096}


def _chunk_cases():
    out = []
    for cfg, c in CHUNKS.items():
        depth = c.bit_length() - 1
        for dt in DTYPES:
            out += [(cfg, dt, c, depth, "one chunk, all its levels"),
                    (cfg, dt, 3 * c + 777, 5, "ragged last chunk"),
                    (cfg, dt, 3 * c + 777, int(np.ceil(np.log2(3 * c + 777))), "ragged, full depth"),
                    (cfg, dt, 65536, 16, "deep: finish kernel / ancestor walk")]
    return out


@pytest.mark.parametrize("cfg,dt,n,L,what", _chunk_cases(), ids=lambda v: str(v))
def test_chunk_configs(T, cfg, dt, n, L, what):
    """Every chunk configuration, forced for the plain calls, against the oracle."""
    from paper_1002_2184_amd import _abi
    assert _abi.haar_force_config_1d(dt, cfg) == 0
    try:
        _check_fwd_inv(T, dt, n, L, seed=1000 + 7 * cfg + n + L, what=f"chunk config {cfg} ({what})")
    finally:
        assert _abi.haar_force_config_1d(dt, -1) == 0


@pytest.mark.parametrize("batch,n,L", [(1, 65536, 16), (3, 65536, 16), (8, 8192, 13), (5, 1 << 18, 18),
                                       (2, 16384, 14), (100, 8192, 13)])
def test_deep_fp32_batches(T, batch, n, L):
    """Deep FP32 analyses (chunks, then the finishing kernel) of batches with
    few and many chunks, including the 1024-sample chunks chosen for
    latency-bound signals: every coefficient against the oracle, on three
    calls in a row and under graph replay with eager calls in between."""
    import torch
    rng = np.random.default_rng(n + L + batch)
    xs = rng.standard_normal((batch, n)).astype(np.float32)
    ref = oracle.fwd_1d(xs.astype(np.float64), L)
    xd = to_device(xs, G.F32)

    def check(y, what):
        yw = to_host(y, G.F32).astype(np.float64)
        for b in range(batch):
            check_signal(yw[b], ref[b], rms(xs[b]), G.F32, f"{what} n={n} L={L} item {b}")
    for rep in range(3):
        check(T.fwd1d(xd, L), f"call {rep}")
    out = torch.empty_like(xd)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        T.fwd1d(xd, L, out=out)
        with torch.cuda.graph(g, stream=side):
            T.fwd1d(xd, L, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        check(out, f"replay {rep}")
        check(T.fwd1d(xd, L), f"eager between replays {rep}")
