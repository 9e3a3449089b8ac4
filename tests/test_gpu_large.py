"""Tensors beyond 2^31 elements (64-bit indexing everywhere).

A tile, chunk or 3D tile whose origin is a multiple of 2^L is its own
subtree of the transform, so an aligned block taken from a huge input can be
checked on its own: its coefficients in the huge output (at the block's
positions in every band) must equal the oracle's transform of the block.
Blocks are taken at the far end of the tensor, where element offsets exceed
2^31.  The round trip is checked on the whole tensor on the GPU."""
import numpy as np
import pytest

import oracle
from gpu_util import FP32_TOL

pytestmark = pytest.mark.gpu

BIG = 2 ** 31


def _item_rms(x) -> float:
    """RMS of the whole input tensor (one item): the scale of the 1e-5 gate."""
    import torch
    return float(torch.linalg.vector_norm(x, dtype=torch.float64)) / float(x.numel()) ** 0.5


def _roundtrip_ok(x, z, scale):
    err = float((z - x).abs().max())
    assert err <= FP32_TOL * scale, f"round trip max err {err:.3e} vs RMS {scale:.3e}"


def test_2d_beyond_2_31_elements():
    import torch
    from paper_1002_2184_amd import transform as T
    H, W, L = 32768, 65600, 5                  # 2.15e9 elements, 8.6 GB in FP32
    assert H * W > BIG
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn(H, W, device="cuda", generator=g)
    scale = _item_rms(x)
    y = T.fwd2d(x, L)
    for (bi, bj) in [(H // 32 - 1, W // 32 - 1), (H // 32 - 1, 3), (700, W // 32 - 2)]:
        blk = x[bi * 32:(bi + 1) * 32, bj * 32:(bj + 1) * 32].double().cpu().numpy()
        ref = oracle.fwd_2d(blk, L)            # the block's own 5-level transform (32 x 32 packed)
        for j in range(1, L + 1):
            s = 32 >> j
            hs, ws = H >> j, W >> j
            r0, c0 = bi * s, bj * s
            got_hl = y[r0:r0 + s, ws + c0:ws + c0 + s]
            got_lh = y[hs + r0:hs + r0 + s, c0:c0 + s]
            got_hh = y[hs + r0:hs + r0 + s, ws + c0:ws + c0 + s]
            for got, want in ((got_hl, ref[:s, s:2 * s]), (got_lh, ref[s:2 * s, :s]), (got_hh, ref[s:2 * s, s:2 * s])):
                err = np.max(np.abs(got.double().cpu().numpy() - want))
                assert err <= FP32_TOL * scale, f"block ({bi},{bj}) level {j}: {err:.3e}"
        ll = y[bi, bj].item()
        assert abs(ll - ref[0, 0]) <= FP32_TOL * scale
    z = T.inv2d(y, L)
    del y
    _roundtrip_ok(x, z, scale)


def test_1d_beyond_2_31_elements():
    import torch
    from paper_1002_2184_amd import transform as T
    n, L = BIG + 8192 + 4096, 12               # 3 chunks past 2^31, 12 levels (one pass)
    g = torch.Generator(device="cuda").manual_seed(8)
    x = torch.randn(n, device="cuda", generator=g)
    scale = _item_rms(x)
    y = T.fwd1d(x, L)
    ns = oracle.sizes_1d(n, L)
    for c in [n // 4096 - 1, n // 4096 - 3, 5]:
        blk = x[c * 4096:(c + 1) * 4096].double().cpu().numpy()
        ref = oracle.fwd_1d(blk, L)            # [a_12 | d_12 | d_11 | ... | d_1] of the chunk
        assert abs(y[c].item() - ref[0]) <= FP32_TOL * scale
        for j in range(1, L + 1):
            s = 4096 >> j
            got = y[ns[j] + c * s:ns[j] + (c + 1) * s].double().cpu().numpy()
            want = ref[s:2 * s]
            assert np.max(np.abs(got - want)) <= FP32_TOL * scale, f"chunk {c} level {j}"
    z = T.inv1d(y, L)
    del y
    _roundtrip_ok(x, z, scale)


def test_3d_beyond_2_31_elements():
    import torch
    from paper_1002_2184_amd import transform as T
    D, H, W, L = 1024, 1024, 2056, 3           # 2.16e9 elements
    assert D * H * W > BIG
    g = torch.Generator(device="cuda").manual_seed(9)
    x = torch.randn(D, H, W, device="cuda", generator=g)
    scale = _item_rms(x)
    y = T.fwd3d(x, L)
    for (bz, by, bx) in [(D // 8 - 1, H // 8 - 1, W // 8 - 1), (D // 8 - 1, 2, W // 8 - 3)]:
        blk = x[bz * 8:(bz + 1) * 8, by * 8:(by + 1) * 8, bx * 8:(bx + 1) * 8].double().cpu().numpy()
        ref = oracle.fwd_3d(blk, L)
        sl = oracle.band_slices_3d(8, 8, 8, L)
        gsl = oracle.band_slices_3d(D, H, W, L)
        for key, (zs, ys, xs) in sl.items():
            gz, gy, gx = gsl[key]
            j = L if key == "LLL" else key[1]
            s = 8 >> j
            oz, oy, ox = gz.start + bz * s, gy.start + by * s, gx.start + bx * s
            n_z, n_y, n_x = zs.stop - zs.start, ys.stop - ys.start, xs.stop - xs.start
            got = y[oz:oz + n_z, oy:oy + n_y, ox:ox + n_x].double().cpu().numpy()
            err = np.max(np.abs(got - ref[zs, ys, xs]))
            assert err <= FP32_TOL * scale, f"block {(bz, by, bx)} band {key}: {err:.3e}"
    z = T.inv3d(y, L)
    del y
    _roundtrip_ok(x, z, scale)
