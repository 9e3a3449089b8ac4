"""Closed forms of the Haar transform used to pin the oracle (test helpers).

Nothing here calls the oracle or the GPU library.  Each builder writes the
transform matrix W (packed output index x input index) from an explicit,
non-recursive description:

* ``haar_matrix_1d_dyadic``: the textbook Haar basis for n divisible by 2^L.
  Row of a_L[k] is 2^(-L/2) on [k 2^L, (k+1) 2^L); row of d_j[k] is 2^(-j/2)
  times -1 on the first half of [k 2^j, (k+1) 2^j) and +1 on the second half
  (the sign follows d = (x1 - x0)/sqrt2, Sec. II listing / Eq. (12)).
* ``carry_matrix_1d``: any n.  The ancestor of x_i at level j is i >> j; it
  is carried (passed unscaled) at level l when it is the last element of an
  odd-length level.  The weight of x_i in a_j[k] is 2^(-c/2), c = number of
  levels 1..j at which x_i's ancestor was paired rather than carried.
* ``haar_matrix_2d_dyadic``: products of 1D scaling/wavelet functions at the
  same scale (separable non-standard decomposition), bands placed in the
  packed quadrant layout.
* ``golden_cases`` / ``paper_coefficients``: parse the hand-derived fixtures.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
R2 = 1.0 / np.sqrt(2.0)


def sizes(n: int, levels: int):
    out = [int(n)]
    for _ in range(levels):
        out.append((out[-1] + 1) // 2)
    return out


def max_levels(n: int) -> int:
    """ceil(log2 n): the depth after which every further level is a no-op."""
    L = 0
    while (1 << L) < n:
        L += 1
    return L


def haar_matrix_1d_dyadic(n: int, L: int) -> np.ndarray:
    assert n % (1 << L) == 0
    W = np.zeros((n, n))
    nL = n >> L
    for k in range(nL):
        W[k, k << L:(k + 1) << L] = 2.0 ** (-L / 2)
    for j in range(1, L + 1):
        nj = n >> j
        half = 1 << (j - 1)
        for k in range(nj):
            start = k << j
            W[nj + k, start:start + half] = -(2.0 ** (-j / 2))
            W[nj + k, start + half:start + 2 * half] = 2.0 ** (-j / 2)
    return W


def _approx_weight(ns, j: int, k: int, i: int) -> float:
    if (i >> j) != k:
        return 0.0
    paired = 0
    for lv in range(1, j + 1):
        p = i >> (lv - 1)
        carried = (ns[lv - 1] % 2 == 1) and (p == ns[lv - 1] - 1)
        if not carried:
            paired += 1
    return 2.0 ** (-paired / 2)


def carry_matrix_1d(n: int, L: int) -> np.ndarray:
    ns = sizes(n, L)
    W = np.zeros((n, n))
    for k in range(ns[L]):
        for i in range(n):
            W[k, i] = _approx_weight(ns, L, k, i)
    for j in range(1, L + 1):
        for k in range(ns[j - 1] // 2):
            row = ns[j] + k
            for i in range(n):
                p = i >> (j - 1)
                if p == 2 * k:
                    W[row, i] = -R2 * _approx_weight(ns, j - 1, 2 * k, i)
                elif p == 2 * k + 1:
                    W[row, i] = R2 * _approx_weight(ns, j - 1, 2 * k + 1, i)
    return W


def _phi(n, j, k):
    v = np.zeros(n)
    v[k << j:(k + 1) << j] = 2.0 ** (-j / 2)
    return v


def _psi(n, j, k):
    v = np.zeros(n)
    s = k << j
    h = 1 << (j - 1)
    v[s:s + h] = -(2.0 ** (-j / 2))
    v[s + h:s + 2 * h] = 2.0 ** (-j / 2)
    return v


def haar_matrix_2d_dyadic(h: int, w: int, L: int) -> np.ndarray:
    """W2 with W2 @ x.ravel() = packed 2D transform of x (h, w divisible by 2^L)."""
    assert h % (1 << L) == 0 and w % (1 << L) == 0
    W = np.zeros((h * w, h * w))

    def put(r, c, vy, vx):
        W[r * w + c] = np.outer(vy, vx).ravel()

    hL, wL = h >> L, w >> L
    for p in range(hL):
        for q in range(wL):
            put(p, q, _phi(h, L, p), _phi(w, L, q))
    for j in range(1, L + 1):
        hj, wj = h >> j, w >> j
        for p in range(hj):
            for q in range(wj):
                put(p, wj + q, _phi(h, j, p), _psi(w, j, q))        # HL: high along width
                put(hj + p, q, _psi(h, j, p), _phi(w, j, q))        # LH: high along height
                put(hj + p, wj + q, _psi(h, j, p), _psi(w, j, q))   # HH
    return W


def _value(tok: str) -> float:
    return float(eval(tok, {"__builtins__": {}}, {"r2": R2}))


def golden_cases():
    """Parse golden/worked_examples.txt into a list of dicts."""
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "worked_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest}
            elif key == "kind":
                cur["kind"] = rest
            elif key == "shape":
                cur["shape"] = tuple(int(t) for t in rest.split())
            elif key == "levels":
                cur["levels"] = int(rest)
            elif key in ("input", "output"):
                cur[key] = np.array([_value(t) for t in rest.split()]).reshape(cur["shape"])
            elif key == "end":
                cases.append(cur)
                cur = None
    return cases


def paper_coefficients():
    out = {}
    with open(os.path.join(GOLDEN, "paper_coefficients.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":")
            vals = []
            for t in rest.split():
                sign = -1.0 if t.startswith("-") else 1.0
                t = t.lstrip("-")
                vals.append(sign * (R2 if t == "r2" else float(t)))
            out[key.strip()] = np.array(vals)
    return out


def poly_mul(a, b):
    return np.convolve(np.asarray(a, float), np.asarray(b, float))


def modulate(h):
    """Taps of H(-z): h[n] (-1)^n."""
    h = np.asarray(h, float)
    return h * ((-1.0) ** np.arange(len(h)))
