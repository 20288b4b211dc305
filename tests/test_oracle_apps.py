"""Pins of the oracle's histogram and piecewise-linear interpolation (the uses of
Sec. 2) against facts fixed by their definitions.

CPU only.  Histogram: a hand-counted example, brute-force counting on tiny
arrays, and conservation of the sample count.  Interpolation: the knots are
reproduced exactly, constant extrapolation outside [X_0, X_N), NaN in gives NaN
out, and the same-precision formula stays within a few rounding errors of the
exact rational interpolant.
"""
import numpy as np

import oracle
import workloads as W
from oracle import apps
from test_oracle import _queries_for, _random_tiny


def test_histogram_hand_example():
    X = np.array([0.0, 1.0, 2.0, 4.0], np.float64)  # N = 3: bins (-inf,0) [0,1) [1,2) [2,4) [4,inf)
    z = np.array([-1.0, 0.0, 0.5, 1.0, 1.5, 1.99, 2.0, 3.0, 4.0, 5.0, np.nan, np.inf, -np.inf])
    assert list(apps.histogram(X, z)) == [3, 2, 3, 2, 3]


def test_histogram_brute_force_and_conservation():
    rng = np.random.default_rng(1)
    for dt in (np.float32, np.float64):
        for n in (1, 2, 5, 17, 64):
            X = _random_tiny(rng, n, dt)
            z = _queries_for(X, rng, m=3000)
            h = apps.histogram(X, z)
            assert h.size == n + 2 and h.sum() == z.size
            for b in range(n + 2):
                lo = -np.inf if b == 0 else X[b - 1]
                hi = np.inf if b == n + 1 else X[b]
                inside = (z >= lo) & (z < hi) if b > 0 else ((z < hi) | np.isnan(z))
                if b == n + 1:
                    inside = z >= lo
                assert h[b] == int(inside.sum()), (n, b)


def test_interp_knots_extrapolation_and_nan():
    rng = np.random.default_rng(2)
    for dt in (np.float32, np.float64):
        X = _random_tiny(rng, 50, dt)
        Y = rng.normal(0, 3, X.size).astype(dt)
        y = apps.interp_linear(X, Y, X[:-1])
        assert np.array_equal(y, Y[:-1])  # t = 0 at every knot but the last
        assert apps.interp_linear(X, Y, X[-1:])[0] == Y[-1]
        out = apps.interp_linear(X, Y, np.array([X[0] - 1, -np.inf, X[-1] + 1, np.inf, np.nan], dt))
        assert out[0] == Y[0] and out[1] == Y[0] and out[2] == Y[-1] and out[3] == Y[-1] and np.isnan(out[4])


def test_interp_within_rounding_of_the_exact_interpolant():
    """Four roundings (two subtractions, the division, the product) and the final sum:
    the error is a few ulps of max(|Y_i|, |Y_{i+1}|) in the array's precision."""
    rng = np.random.default_rng(3)
    for dt in (np.float32, np.float64):
        X = _random_tiny(rng, 40, dt)
        Y = rng.normal(0, 10, X.size).astype(dt)
        z = W.uniform_queries(X[0], X[-1], 3000, np.dtype(dt), rng)
        got = apps.interp_linear(X, Y, z)
        ex = apps.interp_linear_exact(X, Y, z)
        i = oracle.search(X, z)
        eps = float(np.finfo(dt).eps)
        for k in range(z.size):
            scale = max(abs(float(Y[i[k]])), abs(float(Y[i[k] + 1])))
            assert abs(float(got[k]) - float(ex[k])) <= 6 * eps * scale + 1e-300


def test_interp_reproduces_a_line():
    """Knots on y = 3x - 1 (exact in the dtype): the interpolant is the line itself."""
    for dt in (np.float32, np.float64):
        X = np.arange(0, 65, dtype=dt)
        Y = (3 * X - 1).astype(dt)
        z = np.linspace(0, 63.999, 5000).astype(dt)
        got = apps.interp_linear(X, Y, z).astype(np.float64)
        assert np.max(np.abs(got - (3 * z.astype(np.float64) - 1))) <= 8 * float(np.finfo(dt).eps) * 200
