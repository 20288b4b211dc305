"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here runs on a GPU.  The oracle's search is pinned to brute force, to a
library routine and to the defining invariant; its Direct build is pinned to
the paper's worked examples, the infeasible examples, the table identity,
exhaustive enumeration of a float domain, a special case where the two forms
coincide, and the published statistics of the H updates.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _in_domain(X, z, idx):
    """X_i <= z < X_{i+1} for every in-domain query (Sec. 2)."""
    inside = (z >= X[0]) & (z < X[-1])
    i = idx[inside].astype(np.int64)
    zz = z[inside]
    return bool(np.all(i >= 0) and np.all(i < X.size - 1) and np.all(X[i] <= zz) and np.all(zz < X[i + 1]))


def _random_tiny(rng, n, dt):
    return W.gap_array(n, dt, rng, lo=rng.uniform(0.01, 1.0), hi=rng.uniform(1.0, 3.0), x0=rng.uniform(-5, 5))


def _queries_for(X, rng, m=256):
    dt = X.dtype
    lo, hi = float(X[0]), float(X[-1])
    z = rng.uniform(lo - 1, hi + 1, size=m).astype(dt)
    extra = [X, W.prev_float(X, dt), np.nextafter(X, dt.type(np.inf)),
             np.array([np.nan, np.inf, -np.inf, -0.0, 0.0], dt)]
    return np.concatenate([z, *extra]).astype(dt)


# ---------------------------------------------------------------------------
# the result (Sec. 2; classic binary search of Sec. 3.1)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_search_matches_brute_force_on_tiny_arrays(dt):
    rng = np.random.default_rng(11)
    for n in list(range(1, 20)) + [31, 32, 33, 63, 64]:
        X = _random_tiny(rng, n, dt)
        z = _queries_for(X, rng)
        assert np.array_equal(oracle.search(X, z), oracle.brute(X, z)), n


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_search_matches_library_upper_bound(dt):
    rng = np.random.default_rng(12)
    for n in (1, 2, 7, 100, 1000, 4097, 100_000):
        X = _random_tiny(rng, n, dt)
        z = _queries_for(X, rng, m=50_000)
        z = z[~np.isnan(z)]
        expect = np.searchsorted(X, z, side="right") - 1
        got = oracle.search(X, z)
        assert np.array_equal(got, expect.astype(np.int32)), n
        assert _in_domain(X, z, got)


def test_search_adversarial_families_and_outside():
    c = W.plain_f32_1024()
    n = c.N
    assert np.array_equal(oracle.search(c.X, c.z_hits), np.arange(n, dtype=np.int32))
    assert np.array_equal(oracle.search(c.X, c.z_below), np.arange(0, n, dtype=np.int32))
    out = oracle.search(c.X, c.z_outside)
    # nextafter(X_0,-inf), X_N, above X_N, -1e30, 1e30, +inf, -inf, NaN, -0.0 (= X_0)
    assert out.tolist() == [-1, n, n, -1, n, n, -1, -1, 0]
    idx = oracle.search(c.X, c.z_uniform)
    assert _in_domain(c.X, c.z_uniform, idx)


def test_search_thread_count_does_not_change_result():
    X = W.sweep_array(4096, np.float64)
    z = W.sweep_queries(200_000, np.float64)
    assert np.array_equal(oracle.search(X, z, nthreads=1), oracle.search(X, z, nthreads=7))


# ---------------------------------------------------------------------------
# the Direct build (Sec. 4; ComputeHR of Sec. 4.4.3; InitK; FMA form of Sec. 4.9)


def _f_numpy(X, H, W_, form):
    """The grid map evaluated independently with numpy in the array's precision."""
    dt = X.dtype
    H = dt.type(H)
    if form == oracle.FORM_SUB:
        with np.errstate(over="ignore"):
            return np.floor(H * (X - X[0])).astype(np.int64)
    # fma(H, x, -W) via exact rational arithmetic for the product, rounded once
    from fractions import Fraction
    out = []
    for x in X:
        exact = Fraction(float(H)) * Fraction(float(x)) - Fraction(float(W_))
        out.append(int(np.floor(dt.type(float(exact)))) if dt == np.float64 else int(np.floor(np.float32(float(exact)))))
    return np.array(out, np.int64)


def _check_table_invariants(X, t):
    N = X.size - 1
    K = t.K
    assert t.R >= N and t.R < 2**31
    assert K.size == t.R - t.jmin + 1
    assert K[0] == 0 and K[-1] == N
    assert np.all(np.diff(K) >= 0) and np.all(np.diff(K) <= 1)
    fx = _f_numpy(X, t.H, t.W, t.form) if (X.size < 5000 or t.form == oracle.FORM_SUB) else None
    if fx is not None:
        # eq. (cond2): f strictly increasing over X, f(X_0) = jmin, f(X_N) = R
        assert np.all(np.diff(fx) > 0)
        assert fx[0] == t.jmin and fx[-1] == t.R
        # eq. (kidentity): K at f(X_i) is i
        assert np.array_equal(K[fx - t.jmin], np.arange(N + 1))


def test_worked_example_of_section_4_1():
    g = _golden("paper_worked_example.json")
    X = np.array(g["X"], np.float64)
    # the paper's admissible H = 3 gives f(X) = [0, 1, 2, 3]; eq. (indexdef) then gives K = [0, 1, 2, 3]
    H3 = g["H_admissible"]
    st, K = oracle.init_k(X, H3, 0.0, 3, 0)
    assert st == oracle.OK and K.tolist() == [0, 1, 2, 3]
    z = np.array([0.0, 0.1, 0.49, 0.5, 0.6, 0.7, 0.9, 1.0, np.nextafter(1.1, 0)])
    t3 = oracle.DirectTables(oracle.OK, H3, 0.0, 3, 0, 0, K, oracle.FORM_SUB, X.dtype)
    assert np.array_equal(oracle.direct(X, t3, z), oracle.brute(X, z))
    # ComputeHR starts just above 1 / min gap (eq. (minh)) and stays below the
    # eq. (rhtheory) value the paper prints (about 6.36)
    t = oracle.build_direct(X)
    assert t.status == oracle.OK and t.n_updates == 0
    min_gap = np.min(np.diff(X))
    assert t.H > 1.0 / min_gap and t.H < g["H_from_rhtheory_approx"]
    assert t.H == np.nextafter(1.0 / (0.7 - 0.5), np.inf)
    _check_table_invariants(X, t)
    assert np.array_equal(oracle.direct(X, t, z), oracle.brute(X, z))
    # f32 gives the same grid cells
    t32 = oracle.build_direct(X.astype(np.float32))
    assert np.array_equal(t32.K, t.K)


def test_infeasible_examples_of_section_4_4():
    g = _golden("paper_infeasible.json")
    for case in g["cases"]:
        X = np.array(case["X"], np.float32)
        assert strictly(X)
        for form in (oracle.FORM_SUB, oracle.FORM_FMA):
            assert oracle.compute_hr(X, form).status == oracle.ERR_INFEASIBLE, case
    # the second example depends on denormals being kept: 1.42e-45 is a denormal f32
    assert np.float32(1.42e-45) > 0


def strictly(X):
    return bool(np.all(X[1:] > X[:-1]))


def test_rejects_bad_input():
    for dt in (np.float32, np.float64):
        assert oracle.compute_hr(np.array([0, 1, 1, 2], dt)).status == oracle.ERR_NOT_SORTED
        assert oracle.compute_hr(np.array([0, 2, 1], dt)).status == oracle.ERR_NOT_SORTED
        assert oracle.compute_hr(np.array([0, np.nan, 1], dt)).status == oracle.ERR_NONFINITE
        assert oracle.compute_hr(np.array([0, 1, np.inf], dt)).status == oracle.ERR_NONFINITE
    # overflow of R beyond 2^31 (eq. (overflowexact)): range / min gap ~ 1e12
    X = np.array([0.0, 1e-12, 1.0], np.float64)
    assert oracle.compute_hr(X).status == oracle.ERR_INFEASIBLE


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 2, 3, 16, 256, 1024, 4096])
def test_table_invariants_and_direct_equals_search(dt, n):
    rng = np.random.default_rng(n)
    for form in (oracle.FORM_SUB, oracle.FORM_FMA):
        for _ in range(3):
            X = _random_tiny(rng, n, dt)
            t = oracle.build_direct(X, form)
            assert t.status == oracle.OK
            _check_table_invariants(X, t)
            assert t.jmin in ((0,) if form == oracle.FORM_SUB else (-1, 0))
            z = _queries_for(X, rng, m=20_000)
            assert np.array_equal(oracle.direct(X, t, z), oracle.search(X, z))


def test_fma_form_reduces_to_subtraction_form_when_x0_is_zero():
    for dt in (np.float32, np.float64):
        for n in (16, 4096, 65536):
            X = W.sweep_array(n, dt)
            assert X[0] == 0
            a = oracle.build_direct(X, oracle.FORM_SUB)
            b = oracle.build_direct(X, oracle.FORM_FMA)
            assert b.W == 0 and a.H == b.H and a.R == b.R and a.jmin == b.jmin == 0
            assert np.array_equal(a.K, b.K)


def _float_span(lo, count, dt):
    """count consecutive floats of dtype starting at lo."""
    it = np.int32 if dt == np.float32 else np.int64
    base = np.array([lo], dt).view(it)[0]
    return (base + np.arange(count, dtype=it)).view(dt)


@pytest.mark.parametrize("form", [oracle.FORM_SUB, oracle.FORM_FMA])
@pytest.mark.parametrize("start", [1.0, 1000.0, 1.0e-30])
def test_exhaustive_f32_domain(form, start):
    """Every f32 z in [X_0, X_N) for X inside a span of 2^22 consecutive floats."""
    dt = np.float32
    span = _float_span(dt(start), 1 << 22, dt)
    rng = np.random.default_rng(int(start * 7) % 1000 + form)
    pick = np.sort(rng.choice(span.size - 2, size=300, replace=False)) + 1
    X = np.concatenate([[span[0]], span[pick], [span[-1]]]).astype(dt)
    t = oracle.build_direct(X, form)
    assert t.status == oracle.OK
    _check_table_invariants(X, t)
    z = span[:-1]
    got = oracle.direct(X, t, z)
    assert np.array_equal(got, oracle.search(X, z))
    assert np.array_equal(got, (np.searchsorted(X, z, side="right") - 1).astype(np.int32))


def test_dense_neighbourhoods_across_zero():
    """All floats within 2^16 ulps of each X_i and of zero, for X across the sign change."""
    for dt in (np.dtype(np.float32), np.dtype(np.float64)):
        X = np.array([-1.5, -0.7, -0.25, 0.0, 0.3, 0.31, 1.2], dt)
        pts = [*X, dt.type(0.0)]
        z = np.concatenate([np.concatenate([_float_span(p, 1 << 16, dt), -_float_span(-p, 1 << 16, dt)])
                            if p != 0 else np.concatenate([_float_span(dt.type(0), 1 << 16, dt),
                                                           -_float_span(dt.type(0), 1 << 16, dt)])
                            for p in pts]).astype(dt)
        for form in (oracle.FORM_SUB, oracle.FORM_FMA):
            t = oracle.build_direct(X, form)
            assert t.status == oracle.OK
            _check_table_invariants(X, t)
            assert np.array_equal(oracle.direct(X, t, z), oracle.brute(X, z))


def test_plain_workload_direct_equals_search_all_queries():
    c = W.plain_f32_1024()
    z = np.concatenate([c.z_all, c.z_outside])
    ref = oracle.search(c.X, z)
    for form in (oracle.FORM_SUB, oracle.FORM_FMA):
        t = oracle.build_direct(c.X, form)
        assert np.array_equal(oracle.direct(c.X, t, z), ref)


def test_h_update_statistics_match_the_paper():
    """Table 'Number of H updates' (Sec. 6.6) with H started at Hbar; fixed seed."""
    g = _golden("table_h_updates.json")
    rng = np.random.default_rng(2024)
    for row in g["rows"]:
        n = row["N"]
        count = 10_000 if n == 15 else 2_000
        for dt, key in ((np.float32, "f32"), (np.float64, "f64")):
            u = np.empty(count)
            for a in range(count):
                gaps = rng.uniform(1.0, 5.0, n)
                X = np.concatenate([[0.0], np.cumsum(gaps)]).astype(dt)
                t = oracle.compute_hr(X, hstart=oracle.HSTART_HBAR)
                assert t.status == oracle.OK
                u[a] = t.n_updates
            ref = row[key]
            assert u.max() <= max(ref["max"], 1)
            # two-sample 3-sigma band on the mean
            se = np.sqrt(ref["sd"] ** 2 / 10_000 + u.std() ** 2 / count)
            assert abs(u.mean() - ref["mean"]) <= 3 * se + 1e-4, (n, key, u.mean())
    # the literal start phi(Hbar) needed no update on the same kind of arrays
    X = np.concatenate([[0.0], np.cumsum(rng.uniform(1, 5, 15))]).astype(np.float32)
    assert oracle.compute_hr(X).n_updates == 0


def test_h_growth_reaches_a_valid_h_when_needed():
    """Arrays where the start value fails: the growth loop must end with cond2 true."""
    rng = np.random.default_rng(77)
    seen = 0
    for a in range(20_000):
        X = np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 5.0, 15))]).astype(np.float32)
        t = oracle.build_direct(X, hstart=oracle.HSTART_HBAR)
        if t.n_updates:
            seen += 1
            _check_table_invariants(X, t)
            z = _queries_for(X, rng, 2000)
            assert np.array_equal(oracle.direct(X, t, z), oracle.search(X, z))
    assert seen > 0



def _rn32(v):
    """A rational rounded to the nearest float32, ties to even (correct single rounding)."""
    from fractions import Fraction
    c = np.float32(float(v))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - v)
        key = (d, int(np.frombuffer(np.float32(cand).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return best[1]


def _separated_f32(X, H, form):
    """eq. (cond2) at H for every pair, evaluated independently in float32: the subtraction
    form with numpy's correctly rounded float32 operations, the FMA form exactly (rationals,
    one rounding), W = RN(H X_0) recomputed for H."""
    from fractions import Fraction
    H = np.float32(H)
    if form == oracle.FORM_SUB:
        f = np.floor(H * (X - X[0]))
    else:
        Wv = H * X[0]
        f = np.array([np.floor(_rn32(Fraction(float(H)) * Fraction(float(x)) - Fraction(float(Wv)))) for x in X])
    return bool(np.all(np.diff(f) > 0))


def _start_h(X, dt):
    """phi(Hbar) of Sec. 4.4.3 from its definition: Hbar = RN(1 / min RN(D_{i+1} - D_i)),
    D_i = RN(X_i - X_0), all in the dtype; phi is the next float up."""
    D = (X - X[0]).astype(dt)
    g = np.min((D[1:] - D[:-1]).astype(dt))
    hbar = (dt.type(1) / g).astype(dt)
    return np.nextafter(hbar, dt.type(np.inf))


@pytest.mark.parametrize("form", [oracle.FORM_SUB, oracle.FORM_FMA])
def test_h_growth_visits_one_fixed_sequence(form):
    """ComputeHR (Sec. 4.4.3) grows H by P, starting at one step of H (phi(H) - H), adding P
    first and doubling it after, never resetting it between pairs, and re-checks every pair
    until none moves.  So the values of H it can stand on form one fixed sequence
    H_0 = phi(Hbar), H_(k+1) = RN(H_k + 2^k P_0), and it leaves H_k only when some pair still
    shares a cell there: the result must be the first H_k at which every pair is separated,
    after exactly k updates.  A reset of P per pair, or doubling before adding, stands on other
    values and fails this on the near-limit arrays below (16 to 23 updates each).  Single
    precision only: the two precisions share one definition in the oracle, and in double
    precision the arrays whose cells coincide through rounding have R above 2^31."""
    dt = np.dtype(np.float32)
    rng = np.random.default_rng(1506 + form)
    checked = 0
    for a in range(1500 if form == oracle.FORM_SUB else 300):
        X = W.near_limit_array(dt, rng, q=int(rng.integers(1, 4)), n_fill=int(rng.integers(0, 40)),
                               offset=bool(a % 2))
        t = oracle.compute_hr(X, form)
        if t.status != oracle.OK or t.n_updates == 0:
            continue
        H, P = _start_h(X, dt), None
        P = np.nextafter(H, dt.type(np.inf)) - H
        for k in range(64):
            if _separated_f32(X, H, form):
                break
            H, P = np.float32(H + P), np.float32(P + P)
        assert (t.n_updates, t.H) == (k, float(H)), (a, t.n_updates, k, t.H, float(H))
        checked += 1
    assert checked >= (100 if form == oracle.FORM_SUB else 30), checked
