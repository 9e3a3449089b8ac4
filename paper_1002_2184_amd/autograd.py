"""torch.autograd.Functions of the transform.

The transform W is orthonormal (W^T W = I), so the vector-Jacobian product of
the analysis is its adjoint W^T = W^{-1}: the backward of the analysis is the
synthesis bank applied to the incoming gradient, and the backward of the
synthesis is the analysis.  Nothing is saved for backward but the level count.
The transform calls make the incoming gradient contiguous when it is not.
"""
from __future__ import annotations

import torch

from . import transform as T


class HaarFwd1D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, levels):
        ctx.levels = int(levels)
        return T.fwd1d(x, levels)

    @staticmethod
    def backward(ctx, g):
        return T.inv1d(g, ctx.levels), None


class HaarInv1D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, levels):
        ctx.levels = int(levels)
        return T.inv1d(y, levels)

    @staticmethod
    def backward(ctx, g):
        return T.fwd1d(g, ctx.levels), None


class HaarFwd2D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, levels):
        ctx.levels = int(levels)
        return T.fwd2d(x, levels)

    @staticmethod
    def backward(ctx, g):
        return T.inv2d(g, ctx.levels), None


class HaarInv2D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, levels):
        ctx.levels = int(levels)
        return T.inv2d(y, levels)

    @staticmethod
    def backward(ctx, g):
        return T.fwd2d(g, ctx.levels), None


class HaarFwd3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, levels):
        ctx.levels = int(levels)
        return T.fwd3d(x, levels)

    @staticmethod
    def backward(ctx, g):
        return T.inv3d(g, ctx.levels), None


class HaarInv3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, levels):
        ctx.levels = int(levels)
        return T.inv3d(y, levels)

    @staticmethod
    def backward(ctx, g):
        return T.fwd3d(g, ctx.levels), None


def haar_fwd1d(x, levels):
    return HaarFwd1D.apply(x, levels)


def haar_inv1d(y, levels):
    return HaarInv1D.apply(y, levels)


def haar_fwd2d(x, levels):
    return HaarFwd2D.apply(x, levels)


def haar_inv2d(y, levels):
    return HaarInv2D.apply(y, levels)


def haar_fwd3d(x, levels):
    return HaarFwd3D.apply(x, levels)


def haar_inv3d(y, levels):
    return HaarInv3D.apply(y, levels)
