"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``pin_*`` takes an oracle object (``oracle.Oracle``: fwd_1d, inv_1d,
direct_fwd_1d, direct_inv_1d, fwd_2d, inv_2d, fwd_3d, inv_3d, l1_grad_2d, filter_taps) and raises
AssertionError when it disagrees.  None of them re-types the oracle's loops:
they compare it with closed forms, hand-derived fixtures, an independent
formulation (the direct filter bank), polynomial identities of the filter
taps, and invariants (orthonormality, Parseval, perfect reconstruction,
locality, adjointness).  ``tests/test_oracle_mutants.py`` runs the same pins
against deliberately broken copies of the oracle to show that a plausible
mistake anywhere in it fails at least one of them.
"""
from __future__ import annotations

import numpy as np

from haar_closed_form import (R2, carry_matrix_1d, golden_cases, haar_matrix_1d_dyadic,
                              haar_matrix_2d_dyadic, max_levels, modulate, paper_coefficients,
                              poly_mul, sizes)

TOL = 1e-13


def _close(a, b, tol=TOL, what=""):
    a, b = np.asarray(a, float), np.asarray(b, float)
    assert a.shape == b.shape, f"{what}: shape {a.shape} != {b.shape}"
    scale = max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    err = float(np.max(np.abs(a - b))) if a.size else 0.0
    assert err <= tol * scale, f"{what}: max err {err:.3e} > {tol:.1e}*{scale:.3g}"


def matrix_1d(orc, n, L, inverse=False):
    """Columns are the transform of unit vectors (one batched call)."""
    eye = np.eye(n)
    out = (orc.inv_1d if inverse else orc.fwd_1d)(eye, L)   # row i = T(e_i)
    return out.T


def matrix_2d(orc, h, w, L, inverse=False):
    eye = np.eye(h * w).reshape(h * w, h, w)
    out = (orc.inv_2d if inverse else orc.fwd_2d)(eye, L)
    return out.reshape(h * w, h * w).T


# ---------------------------------------------------------------------------
def pin_paper_coefficients(orc):
    """Sec. II listings and Eq. (19): one level on n = 2."""
    c = paper_coefficients()
    W = matrix_1d(orc, 2, 1)          # rows: (a, d); columns: (x0, x1)
    _close(W[0], c["lowpass_analysis"], 1e-15, "lowpass analysis taps")
    _close(W[1], c["highpass_analysis"], 1e-15, "highpass analysis taps")
    V = matrix_1d(orc, 2, 1, inverse=True)   # columns: output for a=1 / d=1
    _close(V[:, 0], c["lowpass_synthesis_eq19"], 1e-15, "lowpass synthesis")
    _close(V[:, 1], c["highpass_synthesis_eq19"], 1e-15, "highpass synthesis")
    _close(W[0, 0], c["b00"][0], 1e-15, "b00")


def pin_worked_examples(orc):
    """Hand-derived examples (golden/worked_examples.txt)."""
    for case in golden_cases():
        if case["kind"] == "1d":
            y = orc.fwd_1d(case["input"], case["levels"])
            _close(y, case["output"], 1e-14, case["name"])
            _close(orc.inv_1d(case["output"], case["levels"]), case["input"], 1e-14,
                   case["name"] + " inverse")
        else:
            y = orc.fwd_2d(case["input"], case["levels"])
            _close(y, case["output"], 1e-14, case["name"])
            _close(orc.inv_2d(case["output"], case["levels"]), case["input"], 1e-14,
                   case["name"] + " inverse")


def pin_dyadic_closed_form(orc):
    """Textbook Haar basis for n = 2^K (impulse at 2m -> a=1/sqrt2, d=-1/sqrt2, ...)."""
    for K in range(1, 7):
        n = 1 << K
        for L in range(0, K + 1):
            _close(matrix_1d(orc, n, L), haar_matrix_1d_dyadic(n, L), 1e-14, f"n={n} L={L}")
    for (n, L) in [(24, 3), (40, 2), (48, 4)]:
        _close(matrix_1d(orc, n, L), haar_matrix_1d_dyadic(n, L), 1e-14, f"n={n} L={L}")


def pin_carry_weights(orc):
    """Any length under the carry rule, against the explicit weight formula."""
    for n in range(1, 41):
        for L in range(0, max_levels(n) + 1):
            _close(matrix_1d(orc, n, L), carry_matrix_1d(n, L), 1e-14, f"carry n={n} L={L}")


def pin_carry_impulse(orc):
    """n = 2^L + 1: the last sample is carried at every level, unscaled."""
    for L in range(1, 7):
        n = (1 << L) + 1
        x = np.zeros(n)
        x[-1] = 1.0
        y = orc.fwd_1d(x, L)
        e = np.zeros(n)
        e[sizes(n, L)[L] - 1] = 1.0
        _close(y, e, 0.0, f"carry impulse n={n}")


def pin_orthonormal_and_inverse(orc):
    """W W^T = I; the synthesis matrix is W^T (1D all n <= 33, 2D small)."""
    for n in list(range(1, 34)) + [64]:
        for L in range(0, max_levels(n) + 1):
            W = matrix_1d(orc, n, L)
            _close(W @ W.T, np.eye(n), 1e-14, f"orthonormal n={n} L={L}")
            _close(matrix_1d(orc, n, L, inverse=True), W.T, 1e-14, f"inverse n={n} L={L}")
    for (h, w) in [(1, 1), (1, 5), (4, 1), (3, 3), (5, 7), (8, 8), (6, 10), (9, 4)]:
        for L in range(0, max_levels(max(h, w)) + 1):
            W = matrix_2d(orc, h, w, L)
            _close(W @ W.T, np.eye(h * w), 1e-14, f"2D orthonormal {h}x{w} L={L}")
            _close(matrix_2d(orc, h, w, L, inverse=True), W.T, 1e-14, f"2D inverse {h}x{w} L={L}")


def pin_direct_equals_fast(orc):
    """The direct bank (Fig. 2, convolve then decimate) equals the fast bank (Fig. 4)."""
    rng = np.random.default_rng(7)
    for n in [1, 2, 3, 7, 16, 31, 64, 100, 257, 1024]:
        for L in sorted({0, 1, max_levels(n) // 2, max_levels(n)}):
            x = rng.standard_normal((3, n))
            y = orc.fwd_1d(x, L)
            _close(orc.direct_fwd_1d(x, L), y, 1e-14, f"direct fwd n={n} L={L}")
            _close(orc.direct_inv_1d(y, L), orc.inv_1d(y, L), 1e-14, f"direct inv n={n} L={L}")


def pin_alias_free_taps(orc):
    """Polynomial identities of the direct-structure taps (Eq. (6), (9), (13), (17), (18)).

    T(z) = 1/2 [B0(z)A0(z) + B1(z)A1(z)] = z^-1   (perfect reconstruction, delay 1)
    A(z) = 1/2 [B0(-z)A0(z) + B1(-z)A1(z)] = 0    (alias term cancelled)
    B1(z) = B0(-z)                               (QMF choice, Eq. (6))"""
    b0, b1, a0, a1 = orc.filter_taps()
    T = 0.5 * (poly_mul(b0, a0) + poly_mul(b1, a1))
    A = 0.5 * (poly_mul(modulate(b0), a0) + poly_mul(modulate(b1), a1))
    _close(T, [0.0, 1.0, 0.0], 1e-15, "distortion T(z)")
    _close(A, [0.0, 0.0, 0.0], 1e-15, "alias A(z)")
    _close(b1, modulate(b0), 1e-15, "QMF B1(z)=B0(-z)")
    _close(b0, [R2, R2], 1e-15, "b0 = [b00, b01]")


def pin_constant(orc):
    """Constant c: zero details, a_L = c 2^(L/2) (1D), LL_L = c 2^L (2D) when 2^L | n."""
    c = 3.25
    for (n, L) in [(8, 3), (64, 4), (1024, 10), (96, 5)]:
        y = orc.fwd_1d(np.full(n, c), L)
        nL = n >> L
        _close(y[:nL], np.full(nL, c * 2.0 ** (L / 2)), 1e-15, f"const approx n={n}")
        assert np.all(y[nL:] == 0.0), f"const details n={n}"
    for (h, w, L) in [(8, 8, 3), (32, 64, 5), (48, 16, 4)]:
        y = orc.fwd_2d(np.full((h, w), c), L)
        hL, wL = h >> L, w >> L
        _close(y[:hL, :wL], np.full((hL, wL), c * 2.0 ** L), 1e-15, f"const LL {h}x{w}")
        mask = np.ones((h, w), bool)
        mask[:hL, :wL] = False
        assert np.all(y[mask] == 0.0), f"const 2D details {h}x{w}"


def pin_parseval_and_pr(orc):
    """Energy preservation and perfect reconstruction on random data, odd sizes too."""
    rng = np.random.default_rng(11)
    for n in [5, 64, 1000, 4097]:
        for L in [1, 3, max_levels(n)]:
            x = rng.standard_normal((2, n))
            y = orc.fwd_1d(x, L)
            _close(np.sum(y * y, -1), np.sum(x * x, -1), 1e-13, f"Parseval n={n}")
            _close(orc.inv_1d(y, L), x, 1e-13, f"PR n={n} L={L}")
    for (h, w) in [(7, 9), (64, 48), (130, 66)]:
        for L in [1, 2, max_levels(max(h, w))]:
            x = rng.standard_normal((2, h, w))
            y = orc.fwd_2d(x, L)
            _close(np.sum(y * y, (-1, -2)), np.sum(x * x, (-1, -2)), 1e-13, f"2D Parseval {h}x{w}")
            _close(orc.inv_2d(y, L), x, 1e-13, f"2D PR {h}x{w} L={L}")


def _bands_1d(orc, u, j):
    """(a_j(u), d_j(u)) from a j-level transform of u."""
    ns = sizes(len(u), j)
    y = orc.fwd_1d(u, j)
    return y[:ns[j]], y[ns[j]:ns[j - 1]]


def pin_2d_separable(orc):
    """Rank-1 inputs u v^T: every 2D band is an outer product of 1D bands
    (LL_L = a_L(u) a_L(v)^T, HL_j = a_j(u) d_j(v)^T, LH_j = d_j(u) a_j(v)^T,
    HH_j = d_j(u) d_j(v)^T), odd sizes included; by linearity, unit impulses
    e_p e_q^T pin the whole 2D operator to the 1D one."""
    rng = np.random.default_rng(13)
    shapes = [(1, 1), (1, 6), (5, 1), (3, 3), (5, 7), (8, 8), (12, 10), (17, 9), (33, 20)]
    for (h, w) in shapes:
        for L in range(0, max_levels(max(h, w)) + 1):
            for trial in range(2):
                if trial == 0 and h * w <= 100:
                    p, q = int(rng.integers(h)), int(rng.integers(w))
                    u = np.zeros(h); u[p] = 1.0
                    v = np.zeros(w); v[q] = 1.0
                else:
                    u, v = rng.standard_normal(h), rng.standard_normal(w)
                y = orc.fwd_2d(np.outer(u, v), L)
                hs, ws = sizes(h, L), sizes(w, L)
                exp = np.zeros((h, w))
                if L == 0:
                    exp = np.outer(u, v)
                else:
                    au = orc.fwd_1d(u, L)[:hs[L]]
                    av = orc.fwd_1d(v, L)[:ws[L]]
                    exp[:hs[L], :ws[L]] = np.outer(au, av)
                    for j in range(1, L + 1):
                        aju, dju = _bands_1d(orc, u, j)
                        ajv, djv = _bands_1d(orc, v, j)
                        exp[:hs[j], ws[j]:ws[j - 1]] = np.outer(aju, djv)
                        exp[hs[j]:hs[j - 1], :ws[j]] = np.outer(dju, ajv)
                        exp[hs[j]:hs[j - 1], ws[j]:ws[j - 1]] = np.outer(dju, djv)
                _close(y, exp, 1e-13, f"rank-1 {h}x{w} L={L}")


def pin_2d_dyadic_closed_form(orc):
    """2D Haar basis = products of 1D scaling/wavelet functions at one scale."""
    for (h, w, L) in [(2, 2, 1), (4, 4, 2), (8, 8, 3), (16, 8, 2), (4, 16, 2), (8, 4, 1)]:
        _close(matrix_2d(orc, h, w, L), haar_matrix_2d_dyadic(h, w, L), 1e-14, f"2D basis {h}x{w} L={L}")


def pin_locality(orc):
    """Perturbing one aligned 2^L block changes only its own dyadic subtree."""
    rng = np.random.default_rng(17)
    n, L, blk = 64, 3, 5
    x = rng.standard_normal(n)
    x2 = x.copy()
    x2[blk * 8:(blk + 1) * 8] += rng.standard_normal(8)
    diff = orc.fwd_1d(x2, L) != orc.fwd_1d(x, L)
    expect = np.zeros(n, bool)
    expect[blk] = True                         # a_3[blk]
    expect[8 + blk] = True                     # d_3[blk]
    expect[16 + 2 * blk:16 + 2 * blk + 2] = True   # d_2
    expect[32 + 4 * blk:32 + 4 * blk + 4] = True   # d_1
    assert np.array_equal(diff, expect), "1D locality"
    h, w, L = 32, 48, 3
    X = rng.standard_normal((h, w))
    X2 = X.copy()
    by, bx = 2, 4
    X2[by * 8:(by + 1) * 8, bx * 8:(bx + 1) * 8] += 1.0 + rng.random((8, 8))
    D = orc.fwd_2d(X2, L) != orc.fwd_2d(X, L)
    E = np.zeros((h, w), bool)
    for j in range(1, L + 1):
        s = 8 >> j
        hj, wj = h >> j, w >> j
        r0, c0 = by * s, bx * s
        E[r0:r0 + s, wj + c0:wj + c0 + s] = True
        E[hj + r0:hj + r0 + s, c0:c0 + s] = True
        E[hj + r0:hj + r0 + s, wj + c0:wj + c0 + s] = True
    E[by, bx] = True
    assert np.array_equal(D, E), "2D locality"


def pin_adjoint(orc):
    """<fwd x, g> = <x, inv g> (the backward of the transform is its inverse)."""
    rng = np.random.default_rng(19)
    for n, L in [(37, 4), (256, 8), (1000, 5)]:
        x, g = rng.standard_normal(n), rng.standard_normal(n)
        lhs, rhs = float(orc.fwd_1d(x, L) @ g), float(x @ orc.inv_1d(g, L))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), "1D adjoint"
    for (h, w, L) in [(9, 14, 3), (64, 64, 5)]:
        x, g = rng.standard_normal((h, w)), rng.standard_normal((h, w))
        lhs = float(np.sum(orc.fwd_2d(x, L) * g))
        rhs = float(np.sum(x * orc.inv_2d(g, L)))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), "2D adjoint"


# ---------------------------------------------------------------------------
# Shrinkage (analysis, per-level thresholding of the details, synthesis)
# ---------------------------------------------------------------------------
def _shrink(c, mode, t):
    if mode == 0:
        return np.where(np.abs(c) > t, c, 0.0)
    return np.sign(c) * np.maximum(np.abs(c) - t, 0.0)


def _row_levels_1d(n, L):
    """Level of every packed 1D coefficient (0 for the approximation a_L)."""
    ns = sizes(n, L)
    lev = np.zeros(n, dtype=int)
    for j in range(1, L + 1):
        lev[ns[j]:ns[j - 1]] = j
    return lev


def _row_levels_2d(h, w, L):
    hs, ws = sizes(h, L), sizes(w, L)
    lev = np.zeros((h, w), dtype=int)
    for j in range(L, 0, -1):            # inside the level-(j-1) LL region, outside level j's
        region = np.zeros((h, w), dtype=bool)
        region[:hs[j - 1], :ws[j - 1]] = True
        region[:hs[j], :ws[j]] = False
        lev[region] = j
    return lev.ravel()


def _thresholds_away(coefs, lev, L, rng, margin=1e-6):
    """Per-level thresholds drawn from the spread of each level's magnitudes,
    moved off any coefficient magnitude so that the keep/zero decision is
    unambiguous."""
    t = np.zeros(L)
    for j in range(1, L + 1):
        mags = np.abs(coefs[lev == j])
        while True:
            cand = float(rng.uniform(0.0, 1.2) * (mags.max() if mags.size else 1.0))
            if mags.size == 0 or np.min(np.abs(mags - cand)) > margin * max(cand, 1e-12):
                t[j - 1] = cand
                break
    return t


def pin_shrink_matrix(orc):
    """shrink(x) = W^T S(W x) with W the closed-form transform matrix (any 1D
    length, 2D sizes divisible by 2^L), S the per-level threshold rule."""
    rng = np.random.default_rng(23)
    for n, L in [(16, 4), (13, 3), (33, 5), (24, 2), (7, 3)]:
        W = carry_matrix_1d(n, L)
        lev = _row_levels_1d(n, L)
        for mode in (0, 1):
            x = rng.standard_normal(n)
            c = W @ x
            t = _thresholds_away(c, lev, L, rng)
            tt = np.concatenate([[0.0], t])[lev]
            want = W.T @ np.where(lev > 0, _shrink(c, mode, tt), c)
            _close(orc.shrink_1d(x, L, mode, t), want, 1e-12, f"1D shrink n={n} L={L} mode {mode}")
    for h, w, L in [(8, 8, 3), (4, 8, 2), (16, 8, 3)]:
        W = haar_matrix_2d_dyadic(h, w, L)
        lev = _row_levels_2d(h, w, L)
        for mode in (0, 1):
            x = rng.standard_normal((h, w))
            c = W @ x.ravel()
            t = _thresholds_away(c, lev, L, rng)
            tt = np.concatenate([[0.0], t])[lev]
            want = (W.T @ np.where(lev > 0, _shrink(c, mode, tt), c)).reshape(h, w)
            _close(orc.shrink_2d(x, L, mode, t), want, 1e-12, f"2D shrink {h}x{w} L={L} mode {mode}")


def pin_shrink_extremes(orc):
    """Threshold 0 reconstructs the input; an infinite threshold leaves the
    block means (every aligned 2^L block, or 2^L x 2^L block, replaced by its
    mean, when 2^L divides the size)."""
    rng = np.random.default_rng(29)
    x = rng.standard_normal((2, 96))
    for mode in (0, 1):
        _close(orc.shrink_1d(x, 5, mode, np.zeros(5)), x, TOL, f"1D threshold 0 mode {mode}")
        blocks = x.reshape(2, 96 // 32, 32).mean(axis=-1, keepdims=True)
        want = np.broadcast_to(blocks, (2, 3, 32)).reshape(2, 96)
        _close(orc.shrink_1d(x, 5, mode, np.full(5, 1e300)), want, TOL, f"1D block means mode {mode}")
    x2 = rng.standard_normal((24, 40))
    for mode in (0, 1):
        _close(orc.shrink_2d(x2, 3, mode, np.zeros(3)), x2, TOL, f"2D threshold 0 mode {mode}")
        m = x2.reshape(3, 8, 5, 8).mean(axis=(1, 3))
        want = np.repeat(np.repeat(m, 8, axis=0), 8, axis=1)
        _close(orc.shrink_2d(x2, 3, mode, np.full(3, 1e300)), want, TOL, f"2D block means mode {mode}")


def pin_shrink_hard_projection(orc):
    """Hard thresholding in an orthonormal basis is a projection: applying it
    twice equals applying it once (odd sizes included)."""
    rng = np.random.default_rng(31)
    x = rng.standard_normal((3, 101))
    t = np.array([0.5, 0.8, 1.1, 0.3])
    once = orc.shrink_1d(x, 4, 0, t)
    _close(orc.shrink_1d(once, 4, 0, t), once, 1e-12, "1D hard twice")
    x2 = rng.standard_normal((37, 29))
    t2 = np.array([0.7, 1.0, 1.5])
    once2 = orc.shrink_2d(x2, 3, 0, t2)
    _close(orc.shrink_2d(once2, 3, 0, t2), once2, 1e-12, "2D hard twice")


# ---------------------------------------------------------------------------
# Separable 3D (volumes [d][h][w]; per level x, then y, then z on LLL).


def _bands3_expected(orc, u, v, w, L):
    """Packed 3D transform of the rank-1 volume u (x) v (x) w (z, y, x) from
    1D transforms: band (x, y, z filters) at level j is the outer product of
    a_j or d_j of each factor, LLL_L = a_L(u) a_L(v) a_L(w)."""
    d, h, wd = len(u), len(v), len(w)
    if L == 0:
        return np.einsum("i,j,k->ijk", u, v, w)
    ds, hs, ws = sizes(d, L), sizes(h, L), sizes(wd, L)
    exp = np.zeros((d, h, wd))
    au, av, aw = (orc.fwd_1d(t, L)[:sizes(len(t), L)[L]] for t in (u, v, w))
    exp[:ds[L], :hs[L], :ws[L]] = np.einsum("i,j,k->ijk", au, av, aw)
    for j in range(1, L + 1):
        pu, pv, pw = _bands_1d(orc, u, j), _bands_1d(orc, v, j), _bands_1d(orc, w, j)
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    if bx == by == bz == 0:
                        continue
                    zs = slice(ds[j], ds[j - 1]) if bz else slice(0, ds[j])
                    ys = slice(hs[j], hs[j - 1]) if by else slice(0, hs[j])
                    xs = slice(ws[j], ws[j - 1]) if bx else slice(0, ws[j])
                    exp[zs, ys, xs] = np.einsum("i,j,k->ijk", pu[bz], pv[by], pw[bx])
    return exp


def pin_3d_separable(orc):
    """Rank-1 volumes u (x) v (x) w: every 3D band is an outer product of the
    1D bands of the factors, at every level and for odd sizes (carries on
    each axis); impulses e_p (x) e_q (x) e_r pin the operator entry by entry.
    The inverse maps the expected bands back to the volume."""
    rng = np.random.default_rng(23)
    shapes = [(1, 1, 1), (1, 1, 6), (1, 5, 1), (7, 1, 1), (2, 2, 2), (3, 5, 7), (8, 8, 8),
              (5, 9, 4), (9, 6, 11), (16, 4, 12)]
    for (d, h, w) in shapes:
        for L in range(0, max_levels(max(d, h, w)) + 1):
            for trial in range(2):
                if trial == 0:
                    u, v, t = np.zeros(d), np.zeros(h), np.zeros(w)
                    u[rng.integers(d)] = 1.0
                    v[rng.integers(h)] = 1.0
                    t[rng.integers(w)] = 1.0
                else:
                    u, v, t = rng.standard_normal(d), rng.standard_normal(h), rng.standard_normal(w)
                x = np.einsum("i,j,k->ijk", u, v, t)
                exp = _bands3_expected(orc, u, v, t, L)
                _close(orc.fwd_3d(x, L), exp, 1e-13, f"3D rank-1 {d}x{h}x{w} L={L}")
                _close(orc.inv_3d(exp, L), x, 1e-13, f"3D rank-1 inverse {d}x{h}x{w} L={L}")


def pin_3d_reductions(orc):
    """A volume of depth 1 is an image (the 3D transform reduces to the 2D
    one); a volume of one row and one column is a 1D signal along z."""
    rng = np.random.default_rng(29)
    for (h, w, L) in [(7, 9, 3), (16, 12, 2), (5, 33, 5)]:
        x = rng.standard_normal((2, h, w))
        _close(orc.fwd_3d(x[:, None], L)[:, 0], orc.fwd_2d(x, L), 1e-15, f"3D depth 1 {h}x{w}")
        _close(orc.inv_3d(x[:, None], L)[:, 0], orc.inv_2d(x, L), 1e-15, f"3D inv depth 1 {h}x{w}")
    for (d, L) in [(13, 3), (64, 6)]:
        x = rng.standard_normal((2, d))
        _close(orc.fwd_3d(x[:, :, None, None], L)[:, :, 0, 0], orc.fwd_1d(x, L), 1e-15, f"3D z line {d}")
        _close(orc.inv_3d(x[:, :, None, None], L)[:, :, 0, 0], orc.inv_1d(x, L), 1e-15, f"3D inv z {d}")


def pin_3d_invariants(orc):
    """Constant volumes (2^L | d, h, w): zero details, LLL_L = c 2^(3L/2).
    Orthonormality of the full matrix on small odd volumes; Parseval and
    perfect reconstruction on random volumes."""
    c = -1.75
    for (d, h, w, L) in [(8, 8, 8, 3), (4, 16, 32, 2), (16, 16, 16, 4)]:
        y = orc.fwd_3d(np.full((d, h, w), c), L)
        dL, hL, wL = d >> L, h >> L, w >> L
        _close(y[:dL, :hL, :wL], np.full((dL, hL, wL), c * 2.0 ** (1.5 * L)), 1e-15, "3D const LLL")
        mask = np.ones((d, h, w), bool)
        mask[:dL, :hL, :wL] = False
        assert np.all(y[mask] == 0.0), f"3D const details {d}x{h}x{w}"
    for (d, h, w, L) in [(3, 4, 5, 2), (2, 3, 2, 1), (5, 3, 3, 3)]:
        n = d * h * w
        M = orc.fwd_3d(np.eye(n).reshape(n, d, h, w), L).reshape(n, n).T
        _close(M @ M.T, np.eye(n), 1e-14, f"3D orthonormal {d}x{h}x{w}")
        Mi = orc.inv_3d(np.eye(n).reshape(n, d, h, w), L).reshape(n, n).T
        _close(Mi, M.T, 1e-14, f"3D synthesis = analysis^T {d}x{h}x{w}")
    rng = np.random.default_rng(31)
    for (d, h, w, L) in [(9, 17, 33, 4), (32, 16, 64, 3), (6, 6, 130, 2)]:
        x = rng.standard_normal((2, d, h, w))
        y = orc.fwd_3d(x, L)
        _close(np.sum(y * y, (1, 2, 3)), np.sum(x * x, (1, 2, 3)), 1e-13, "3D Parseval")
        _close(orc.inv_3d(y, L), x, 1e-13, f"3D PR {d}x{h}x{w}")


# ---------------------------------------------------------------------------
# Gradient of the sparsity loss through the 2D transform.


def pin_l1_grad_matrix(orc):
    """With W the closed-form 2D Haar matrix (dyadic sizes) and c = W x:
    loss = sum |c_details| + 0.5 sum c_LL^2 and grad_x = W^T (sign(c_details),
    c_LL)."""
    rng = np.random.default_rng(37)
    for (h, w, L) in [(4, 4, 1), (8, 8, 3), (16, 8, 2), (8, 16, 3)]:
        W = haar_matrix_2d_dyadic(h, w, L)
        x = rng.standard_normal((3, h, w))
        loss, g = orc.l1_grad_2d(x, L)
        ll = np.zeros((h, w), bool)
        ll[:h >> L, :w >> L] = True
        llv = ll.ravel()
        for b in range(3):
            c = W @ x[b].ravel()
            want_loss = np.sum(np.abs(c[~llv])) + 0.5 * np.sum(c[llv] ** 2)
            s = np.where(llv, c, np.sign(c))
            _close(loss[b], want_loss, 1e-13, f"l1 loss {h}x{w} L={L}")
            _close(g[b].ravel(), W.T @ s, 1e-13, f"l1 grad {h}x{w} L={L}")


def pin_l1_grad_finite_differences(orc):
    """Central differences of the oracle's own loss match its gradient on odd
    and even sizes (the loss is smooth away from zero coefficients; indices
    whose step would move a detail across zero are skipped)."""
    rng = np.random.default_rng(41)
    eps = 1e-6
    for (h, w, L) in [(5, 7, 2), (9, 6, 3), (8, 8, 3), (3, 11, 1)]:
        x = rng.standard_normal((h, w))
        loss, g = orc.l1_grad_2d(x, L)
        c = orc.fwd_2d(x, L)
        checked = 0
        for i in rng.permutation(h * w)[:20]:
            e = np.zeros(h * w)
            e[i] = eps
            e = e.reshape(h, w)
            cp, cm = orc.fwd_2d(x + e, L), orc.fwd_2d(x - e, L)
            if np.any(np.sign(cp) != np.sign(c)) or np.any(np.sign(cm) != np.sign(c)):
                continue
            fd = (orc.l1_grad_2d(x + e, L)[0] - orc.l1_grad_2d(x - e, L)[0]) / (2 * eps)
            assert abs(fd - g.ravel()[i]) <= 1e-6 * max(1.0, abs(g.ravel()[i])), \
                f"l1 FD {h}x{w} L={L} index {i}: {fd} vs {g.ravel()[i]}"
            checked += 1
        assert checked >= 10, f"too few FD indices away from kinks ({checked})"


ALL_PINS = [
    pin_paper_coefficients, pin_worked_examples, pin_dyadic_closed_form, pin_carry_weights,
    pin_carry_impulse, pin_orthonormal_and_inverse, pin_direct_equals_fast, pin_alias_free_taps,
    pin_constant, pin_parseval_and_pr, pin_2d_separable, pin_2d_dyadic_closed_form,
    pin_locality, pin_adjoint, pin_shrink_matrix, pin_shrink_extremes, pin_shrink_hard_projection,
    pin_3d_separable, pin_3d_reductions, pin_3d_invariants, pin_l1_grad_matrix,
    pin_l1_grad_finite_differences,
]
