"""Autograd: the backward of the analysis is its adjoint (the synthesis bank).

Workload of the autograd configuration: x ~ N(0,1), [64*3, 512, 512] FP32,
3-level 2D analysis, loss = sum |detail coefficients| + 0.5 * ||LL_3||^2.
Checks: the loss against the FP64 oracle; the gradient against the oracle's
transpose W^T g (same upstream g); central finite differences of the FP64
oracle loss (eps = 1e-3) at 256 seeded indices; the dot-product identity.
"""
import numpy as np
import pytest

import oracle
from gpu_util import rms
from workloads import generators as G

pytestmark = pytest.mark.gpu

L = 3


def _loss_and_upstream(y, L, h, w):
    """sum |details| + 0.5 ||LL_L||^2 of a [..., h, w] coefficient tensor (torch)."""
    import torch
    hL, wL = -(-h // (1 << L)), -(-w // (1 << L))
    mask = torch.ones((h, w), dtype=torch.bool, device=y.device)
    mask[:hL, :wL] = False
    det = y[..., mask]
    ll = y[..., :hL, :wL]
    loss = det.abs().sum() + 0.5 * (ll * ll).sum()
    return loss


def _oracle_block_loss(xb):
    """FP64 loss of one aligned 8x8 block (its coefficients are its own subtree)."""
    c = oracle.fwd_2d(xb, L)
    ll = c[0, 0]
    det = c.copy()
    det[0, 0] = 0.0
    return float(np.sum(np.abs(det)) + 0.5 * ll * ll), c


@pytest.fixture(scope="module")
def cfg4():
    import torch
    from paper_1002_2184_amd import autograd as AG
    x_np = G.config4()
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    y = AG.HaarFwd2D.apply(x, L)
    loss = _loss_and_upstream(y, L, 512, 512)
    (gx,) = torch.autograd.grad(loss, x)
    torch.cuda.synchronize()
    return x_np, y.detach(), float(loss.detach()), gx


def test_loss_matches_oracle(cfg4):
    x_np, _, loss, _ = cfg4
    ref = oracle.fwd_2d(x_np.astype(np.float64), L)
    hL = 512 >> L
    mask = np.ones((512, 512), bool)
    mask[:hL, :hL] = False
    ref_loss = float(np.sum(np.abs(ref[:, mask])) + 0.5 * np.sum(ref[:, :hL, :hL] ** 2))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)


def test_gradient_is_oracle_transpose(cfg4):
    """grad_x = W^T g with g = sign(details) | LL_3, taken from the GPU's own y."""
    x_np, y, _, gx = cfg4
    g = y.clone()
    hL = 512 >> L
    mask = np.ones((512, 512), bool)
    mask[:hL, :hL] = False
    import torch
    m = torch.from_numpy(mask).cuda()
    g[:, m] = torch.sign(y[:, m])
    g64 = g.cpu().numpy().astype(np.float64)
    ref = oracle.inv_2d(g64, L)
    err = float(np.max(np.abs(gx.cpu().numpy().astype(np.float64) - ref)))
    assert err <= 1e-5 * rms(ref), f"max err {err:.3e} vs RMS {rms(ref):.3e}"


def test_finite_differences(cfg4):
    """Central FD of the FP64 oracle loss (eps = 1e-3) at 256 seeded indices,
    evaluated on the aligned 8x8 block containing the index; indices whose
    perturbation flips the sign of a detail coefficient are resampled."""
    x_np, _, _, gx = cfg4
    gx_np = gx.cpu().numpy().astype(np.float64)
    rng = G.rng_for(4, salt=1)
    eps = 1e-3
    checked, skipped = 0, 0
    g_rms = rms(gx_np)
    while checked < 256:
        b, r, c = int(rng.integers(192)), int(rng.integers(512)), int(rng.integers(512))
        r0, c0 = (r // 8) * 8, (c // 8) * 8
        xb = x_np[b, r0:r0 + 8, c0:c0 + 8].astype(np.float64)
        _, coef = _oracle_block_loss(xb)
        e = np.zeros((8, 8))
        e[r - r0, c - c0] = 1.0
        ce = oracle.fwd_2d(e, L)                  # |W_{k,i}| for the kink test
        det = coef.copy()
        det[0, 0] = np.inf
        wk = np.abs(ce)
        wk[0, 0] = 0.0
        if np.any((np.abs(det) < eps * wk) & (wk > 0)):
            skipped += 1
            continue
        xp, xm = xb.copy(), xb.copy()
        xp[r - r0, c - c0] += eps
        xm[r - r0, c - c0] -= eps
        fd = (_oracle_block_loss(xp)[0] - _oracle_block_loss(xm)[0]) / (2 * eps)
        assert abs(gx_np[b, r, c] - fd) <= 1e-5 * g_rms, (b, r, c, gx_np[b, r, c], fd)
        checked += 1
    print(f"FD: 256 indices checked, {skipped} resampled at a kink")


def test_dot_product_identity():
    """<fwd x, g> = <x, inv g> for both autograd directions (FP32 on the GPU)."""
    import torch
    from paper_1002_2184_amd import autograd as AG
    torch.manual_seed(0)
    for shape, lv in (((3, 96, 130), 4), ((2, 512, 512), 3)):
        x = torch.randn(shape, device="cuda", dtype=torch.float64).float()
        g = torch.randn(shape, device="cuda").float()
        lhs = float((AG.HaarFwd2D.apply(x, lv).double() * g.double()).sum())
        rhs = float((x.double() * AG.HaarInv2D.apply(g, lv).double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * float(x.double().norm() * g.double().norm())
    # 1D
    x = torch.randn(4, 5000, device="cuda")
    g = torch.randn(4, 5000, device="cuda")
    lhs = float((AG.HaarFwd1D.apply(x, 13).double() * g.double()).sum())
    rhs = float((x.double() * AG.HaarInv1D.apply(g, 13).double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * float(x.double().norm() * g.double().norm())


def test_backward_of_inverse_and_1d_against_oracle():
    import torch
    from paper_1002_2184_amd import autograd as AG
    rng = np.random.default_rng(21)
    y_np = rng.standard_normal((2, 64, 96)).astype(np.float32)
    g_np = rng.standard_normal((2, 64, 96)).astype(np.float32)
    y = torch.from_numpy(y_np).cuda().requires_grad_(True)
    out = AG.HaarInv2D.apply(y, 4)
    (gy,) = torch.autograd.grad(out, y, torch.from_numpy(g_np).cuda())
    ref = oracle.fwd_2d(g_np.astype(np.float64), 4)          # (W^T)^T g = W g
    assert np.max(np.abs(gy.cpu().numpy() - ref)) <= 1e-5 * rms(ref)
    x_np = rng.standard_normal((3, 4097)).astype(np.float32)
    g1 = rng.standard_normal((3, 4097)).astype(np.float32)
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    (gx,) = torch.autograd.grad(AG.HaarFwd1D.apply(x, 13), x, torch.from_numpy(g1).cuda())
    ref1 = oracle.inv_1d(g1.astype(np.float64), 13)
    assert np.max(np.abs(gx.cpu().numpy() - ref1)) <= 1e-5 * rms(ref1)
