"""Pins of the oracle's gap-q variant (Sec. 4.7, "Relaxing Limitations and
Reducing Memory Usage") against facts fixed by the paper and by mathematics.

CPU only.  The variant only asks f(X_{i+q}) > f(X_i) of the grid (eq.
(f-monotonic-2) for q = 2, eq. (f-monotonic-n) in general), defines
K_j = max{i : f(X_i) <= j} (eq. (kgeneral)) and answers
i = K_j - sum_{k<q} [z < X_{K_j - k}] (eq. (index2), algorithm DirectGap2).
The pins: brute force on tiny arrays for q = 1..4 in both forms, the table
definition evaluated independently with numpy, the two properties of eq.
(kgeneralprop), the grid condition and the lower bound of eq. (fcond11) on H,
the range t - i in {0..q} that the proof of eq. (index2) establishes, the
smaller table that motivates the section, the relaxed feasibility, and
exhaustive enumeration of a float domain.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import _f_numpy, _float_span, _queries_for, _random_tiny


def _k_numpy(fx, jmin, R):
    """eq. (kgeneral) by a library routine: max{i : f(X_i) <= j} = #{i : f(X_i) <= j} - 1."""
    j = np.arange(jmin, R + 1)
    return (np.searchsorted(fx, j, side="right") - 1).astype(np.int32)


def _check_gap_tables(X, t, q):
    N = X.size - 1
    assert t.status == oracle.OK
    assert t.K.size == t.R - t.jmin + 1
    fx = _f_numpy(X, t.H, t.W, t.form)
    assert fx[0] == t.jmin and fx[-1] == t.R
    # the grid condition of eq. (f-monotonic-n)
    assert np.all(fx[q:] > fx[:-q])
    # f non-decreasing (eq. (monotonic))
    assert np.all(np.diff(fx) >= 0)
    # eq. (kgeneral)
    assert np.array_equal(t.K, _k_numpy(fx, t.jmin, t.R))
    assert t.K[-1] == N
    return fx


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_gap_search_matches_brute_force_on_tiny_arrays(dt, q):
    rng = np.random.default_rng(100 + q)
    for n in [q, q + 1, q + 2, 7, 16, 31, 64]:
        if n < q:
            continue
        for form in (oracle.FORM_SUB, oracle.FORM_FMA):
            X = _random_tiny(rng, n, dt)
            t = oracle.build_direct_gap(X, q, form)
            _check_gap_tables(X, t, q)
            z = _queries_for(X, rng, m=2000)
            assert np.array_equal(oracle.direct_gap(X, t, z), oracle.brute(X, z)), (n, form)


def test_kgeneral_properties_for_q2():
    """eq. (kgeneralprop): f(X_i) < f(X_{i+1}) gives K_{f(X_i)} = i; f(X_i) = f(X_{i+1})
    gives K_{f(X_i)} = K_{f(X_{i+1})} = i + 1."""
    rng = np.random.default_rng(5)
    seen_equal = 0
    for dt in (np.float32, np.float64):
        for _ in range(20):
            X = _random_tiny(rng, 200, dt)
            t = oracle.build_direct_gap(X, 2)
            fx = _check_gap_tables(X, t, 2)
            K = t.K
            for i in range(X.size - 2):
                a, b = fx[i], fx[i + 1]
                if a < b:
                    assert K[a - t.jmin] == i
                else:
                    seen_equal += 1
                    assert K[a - t.jmin] == i + 1 and K[b - t.jmin] == i + 1
    assert seen_equal > 0  # the relaxed grid does merge neighbours


@pytest.mark.parametrize("q", [1, 2, 3, 5, 8])
def test_h_bound_and_proof_range(q):
    """H lies above 1 / min_i (X_{i+q} - X_i) (eq. (fcond11)), and t - i is in {0..q} for
    every in-domain query (the three cases of the proof of eq. (index2), generalised)."""
    for dt in (np.float32, np.float64):
        X = W.sweep_array(4096, dt)
        t = oracle.build_direct_gap(X, q)
        _check_gap_tables(X, t, q)
        gq = np.min(X[q:].astype(np.float64) - X[:-q].astype(np.float64))
        assert t.H * gq > 1 - 1e-6
        z = W.sweep_queries(100_000, dt)
        i = oracle.search(X, z).astype(np.int64)
        v = np.floor(np.clip(dt(t.H) * (z - X[0]), t.jmin, t.R)).astype(np.int64)
        tt = t.K[v - t.jmin].astype(np.int64)
        assert np.all((tt - i >= 0) & (tt - i <= q))
        assert np.array_equal(oracle.direct_gap(X, t, z), i.astype(np.int32))


def test_q1_is_plain_directs_grid():
    """For q = 1 the condition is plain Direct's, so ComputeHR gives the same H and R."""
    rng = np.random.default_rng(9)
    for dt in (np.float32, np.float64):
        for form in (oracle.FORM_SUB, oracle.FORM_FMA):
            X = _random_tiny(rng, 500, dt)
            a = oracle.build_direct(X, form)
            b = oracle.build_direct_gap(X, 1, form)
            assert (a.H, a.R, a.jmin, a.n_updates) == (b.H, b.R, b.jmin, b.n_updates)


def test_tables_shrink_with_q():
    """The point of the section: a smaller R.  With gaps U(0.5, 1.5) the minimum q-gap grows
    about linearly in q, so R_q is well below R_1 / q * 2."""
    for dt in (np.float32, np.float64):
        X = W.sweep_array(65536, dt)
        R1 = oracle.compute_hr(X).R
        prev = R1
        for q in (2, 4, 8, 16):
            t = oracle.compute_hr_gap(X, q)
            assert t.status == oracle.OK
            assert t.R <= prev and t.R < 2.0 * R1 / q
            prev = t.R


def test_relaxed_feasibility():
    """Two keys next to each other in [X_0 = -0.5, 0.5], 1e-10 and the next float, have the
    same rounded difference D = m(X - X_0) = 0.5, so no grid separates them and plain Direct is
    infeasible (eq. (distinguishable-exact)); q = 2 only has to separate keys two apart.
    Three such keys defeat q = 2 as well, and q = 3 separates them again."""
    rng = np.random.default_rng(4)
    for dt in (np.float32, np.float64):
        base = (np.cumsum(rng.uniform(0.5, 1.5, 1000)) / 1000.0 - 0.5).astype(dt)
        base = base[np.abs(base) > 1e-3]
        a = dt(1e-10)
        b = np.nextafter(a, dt(np.inf))
        X = np.sort(np.concatenate([[dt(-0.5)], base, [a, b]])).astype(dt)
        assert dt(X[-1] - X[0]) > 0 and (a - X[0]) == (b - X[0])
        assert oracle.compute_hr(X).status == oracle.ERR_INFEASIBLE
        t = oracle.build_direct_gap(X, 2)
        _check_gap_tables(X, t, 2)
        z = np.concatenate([W.uniform_queries(X[0], X[-1], 50_000, np.dtype(dt), rng), X,
                            W.prev_float(X, np.dtype(dt)), [a, b, np.nextafter(b, dt(1))]]).astype(dt)
        assert np.array_equal(oracle.direct_gap(X, t, z), oracle.search(X, z))
        X3 = np.sort(np.concatenate([X, [np.nextafter(b, dt(np.inf))]])).astype(dt)
        assert oracle.compute_hr_gap(X3, 2).status == oracle.ERR_INFEASIBLE
        t3 = oracle.build_direct_gap(X3, 3)
        _check_gap_tables(X3, t3, 3)
        assert np.array_equal(oracle.direct_gap(X3, t3, z), oracle.search(X3, z))


@pytest.mark.parametrize("q", [2, 3])
@pytest.mark.parametrize("form", [oracle.FORM_SUB, oracle.FORM_FMA])
def test_exhaustive_f32_domain_gap(q, form):
    """Every f32 z in [X_0, X_N) for X inside a span of 2^20 consecutive floats."""
    dt = np.float32
    span = _float_span(dt(3.0), 1 << 20, dt)
    rng = np.random.default_rng(q * 10 + form)
    pick = np.sort(rng.choice(span.size - 2, size=400, replace=False)) + 1
    X = np.concatenate([[span[0]], span[pick], [span[-1]]]).astype(dt)
    t = oracle.build_direct_gap(X, q, form)
    _check_gap_tables(X, t, q)
    z = span[:-1]
    assert np.array_equal(oracle.direct_gap(X, t, z), (np.searchsorted(X, z, side="right") - 1).astype(np.int32))


def test_gap_rejects_bad_q():
    X = W.sweep_array(16, np.float32)
    assert oracle.compute_hr_gap(X, 0).status == oracle.ERR_ARG
    assert oracle.compute_hr_gap(X, 17).status == oracle.ERR_ARG
    assert oracle.compute_hr_gap(X, 16).status == oracle.OK
