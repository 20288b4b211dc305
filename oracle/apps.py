"""The two uses of interval search named in Sec. 2, as plain definitions on top of
the oracle's search.

TEST INFRASTRUCTURE ONLY (see the package docstring).

histogram        the number of samples in each interval [X_i, X_{i+1}), plus a bin
                 below X_0 (NaN included) and one at or above X_N: bin i + 1 for
                 search result i, N + 2 bins.
interp_linear    piecewise-linear interpolation of knots (X_i, Y_i), evaluated in
                 the array's precision with numpy (IEEE operations, no contraction)
                 in the order y = Y_i + ((z - X_i) / (X_{i+1} - X_i)) * (Y_{i+1} - Y_i);
                 Y_0 below X_0, Y_N at or above X_N, NaN for NaN.
interp_linear_exact  the same interpolant in exact rational arithmetic (small inputs),
                 for bounding the rounding of the former.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import search


def histogram(X: np.ndarray, z: np.ndarray) -> np.ndarray:
    i = search(X, z).astype(np.int64)
    return np.bincount(i + 1, minlength=X.size + 1).astype(np.int64)


def interp_linear(X: np.ndarray, Y: np.ndarray, z: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X)
    dt = X.dtype
    Y = np.ascontiguousarray(Y, dtype=dt)
    z = np.ascontiguousarray(z, dtype=dt)
    N = X.size - 1
    i = search(X, z).astype(np.int64)
    out = np.empty(z.size, dt)
    below, above = i < 0, i >= N
    mid = ~(below | above)
    out[below] = np.where(np.isnan(z[below]), z[below], Y[0])
    out[above] = Y[N]
    im = i[mid]
    zm = z[mid]
    x0, x1, y0, y1 = X[im], X[im + 1], Y[im], Y[im + 1]
    with np.errstate(all="ignore"):
        t = (zm - x0) / (x1 - x0)
        dy = y1 - y0
        p = t * dy
        out[mid] = y0 + p
    return out


def interp_linear_exact(X: np.ndarray, Y: np.ndarray, z: np.ndarray) -> list:
    """Exact rational value of the interpolant at each in-domain z (None elsewhere)."""
    N = X.size - 1
    i = search(X, z).astype(np.int64)
    res = []
    for k in range(z.size):
        if i[k] < 0 or i[k] >= N:
            res.append(None)
            continue
        a, b = Fraction(float(X[i[k]])), Fraction(float(X[i[k] + 1]))
        ya, yb = Fraction(float(Y[i[k]])), Fraction(float(Y[i[k] + 1]))
        res.append(ya + (Fraction(float(z[k])) - a) / (b - a) * (yb - ya))
    return res
