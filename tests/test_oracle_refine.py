"""Pins of the oracle's H refinement: the bisection of [last infeasible H, grown H]
that the end of Sec. 4.4.3 proposes in place of the grown H of ComputeHR.

CPU only.  Feasibility of an H (eq. (cond2) for q = 1, eq. (f-monotonic-n) for
q > 1, and eq. (overflowexact)) is recomputed here independently of the oracle:
numpy in the array's precision for the subtraction form, exact rationals rounded
once for the FMA form.  Pinned:

* the growth loop's ends: its last infeasible H fails and its final H passes;
* the refined H passes, the float just below it fails, it lies in the growth
  interval, and R does not grow;
* brute force over every float of small intervals: the refined H is the smallest
  feasible float of the interval when feasibility is monotone there, else one of
  its steps from infeasible to feasible;
* at most ceil(log2(floats in the interval)) midpoints are tested;
* the refined tables keep eq. (cond2) and eq. (kidentity), and the search on them
  equals brute force;
* arrays where H never grows, and the paper's own random arrays, where it grows
  by one float, are left unchanged; q = 1 of the gap variant equals plain
  Direct; intervals whose ends are not (infeasible, feasible) are rejected.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import _check_table_invariants, _queries_for

TWO_Q = 2 ** 31


def _rn(fr: Fraction, dt) -> float:
    """fr rounded to nearest-even in dt (Python's int / int division is correctly rounded
    to double; f32 then picks the nearest of three neighbours exactly)."""
    d = fr.numerator / fr.denominator
    if dt == np.float64:
        return d
    c = np.float32(d)
    best = None
    for v in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        err = abs(Fraction(float(v)) - fr)
        key = (err, int(np.array(v).view(np.int32)) & 1)
        if best is None or key < best[0]:
            best = (key, v)
    return float(best[1])


def _grid_floor(X, H, form):
    dt = X.dtype
    if form == oracle.FORM_SUB:
        with np.errstate(over="ignore"):
            return np.floor(dt.type(H) * (X - X[0])).astype(np.float64)
    W_ = _rn(Fraction(float(H)) * Fraction(float(X[0])), dt)
    return np.array([np.floor(_rn(Fraction(float(H)) * Fraction(float(x)) - Fraction(W_), dt)) for x in X])


def _feasible(X, H, q, form):
    f = _grid_floor(X, H, form)
    return bool(f[-1] < TWO_Q) and bool(np.all(f[q:] > f[:-q]))


def _bits(v, dt):
    return int(np.array(v, dt).view(np.int32 if dt == np.float32 else np.int64))


def _prev(v, dt):
    return float(np.nextafter(dt(v), dt(-np.inf)))


def _growth_cases(dt, form, q, count, seed, n_fill=0, offset=False, min_updates=2):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(200 * count):
        X = W.near_limit_array(dt, rng, q=q, n_fill=n_fill, offset=offset)
        if X.size - 1 < q:
            continue
        t = oracle.compute_hr_gap(X, q, form)
        if t.status == oracle.OK and t.n_updates >= min_updates:
            out.append(X)
            if len(out) == count:
                break
    return out


def _check_refined(X, q, form, hstart=oracle.HSTART_PHI):
    dt = X.dtype.type
    g = oracle.compute_hr_gap(X, q, form, hstart)
    r = oracle.compute_hr_gap(X, q, form, hstart, refine=True)
    assert g.status == r.status == oracle.OK and g.n_updates == r.n_updates
    # the growth loop's ends
    assert not _feasible(X, g.H_bad, q, form) and _feasible(X, g.H_grown, q, form)
    assert g.H == g.H_grown == r.H_grown and g.H_bad == r.H_bad
    # the refined H: feasible, predecessor infeasible, inside the interval, R no larger
    assert g.H_bad < r.H <= g.H_grown and r.R <= g.R
    assert _feasible(X, r.H, q, form)
    assert r.H_lo == _prev(r.H, dt) and not _feasible(X, r.H_lo, q, form)
    floats = _bits(g.H_grown, dt) - _bits(g.H_bad, dt)
    assert r.n_refine <= max(0, int(np.ceil(np.log2(floats))))
    if form == oracle.FORM_SUB:
        assert r.W == 0.0
    else:
        assert r.W == _rn(Fraction(r.H) * Fraction(float(X[0])), dt)
    return g, r


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("form", [oracle.FORM_SUB, oracle.FORM_FMA])
def test_refined_h_is_feasible_with_an_infeasible_predecessor(dt, form):
    cases = _growth_cases(dt, form, 1, 40, seed=10 + form, min_updates=1)
    if dt == np.float64:
        # Q = 31 keeps m(H D) below 2^31, far from the ulp of the products, so f64 H grows by one
        # float at most: nothing lies between the ends and the refined H is the grown one
        for X in cases:
            g, r = _check_refined(X, 1, form)
            assert r.H == g.H and r.n_refine == 0
        return
    assert len(cases) == 40
    shrunk = 0
    for X in cases:
        g, r = _check_refined(X, 1, form)
        shrunk += r.R < g.R
    assert shrunk > 10


def test_refined_h_with_an_offset_x0_in_the_fma_form():
    cases = _growth_cases(np.float32, oracle.FORM_FMA, 1, 3, seed=5, offset=True)
    assert cases
    for X in cases:
        _check_refined(X, 1, oracle.FORM_FMA)


def test_refined_tables_and_search():
    rng = np.random.default_rng(7)
    for form in (oracle.FORM_SUB, oracle.FORM_FMA):
        for X in _growth_cases(np.float32, form, 1, 10, seed=20 + form, n_fill=300):
            t = oracle.build_direct(X, form, refine=True)
            assert t.status == oracle.OK and t.n_refine > 0
            _check_table_invariants(X, t)
            z = _queries_for(X, rng, m=2000)
            assert np.array_equal(oracle.direct(X, t, z), oracle.brute(X, z))


def _feasible_many(X, Hs, q):
    """Subtraction-form feasibility of every H in Hs at once (numpy, the array's precision)."""
    D = (X - X[0])[None, :]
    out = np.empty(Hs.size, bool)
    for a in range(0, Hs.size, 1 << 18):
        f = np.floor(Hs[a:a + (1 << 18), None] * D)
        out[a:a + (1 << 18)] = np.all(f[:, q:] > f[:, :-q], axis=1) & (f[:, -1] < TWO_Q)
    return out


def test_brute_force_over_the_interval():
    """Every float of the growth interval is classified; the bisection must stop on a step
    from infeasible to feasible, the first one when there is only one."""
    dt = np.float32
    monotone = 0
    cases = _growth_cases(dt, oracle.FORM_SUB, 1, 12, seed=30)
    assert len(cases) == 12
    for X in cases:
        g = oracle.compute_hr(X)
        lo, hi = _bits(g.H_bad, dt), _bits(g.H_grown, dt)
        Hs = np.arange(lo, hi + 1, dtype=np.int32).view(np.float32)
        ok = _feasible_many(X, Hs, 1)
        assert not ok[0] and ok[-1]
        assert ok[-1] == _feasible(X, g.H_grown, 1, oracle.FORM_SUB)
        steps = np.flatnonzero(~ok[:-1] & ok[1:]) + 1
        r = oracle.compute_hr(X, refine=True)
        k = _bits(r.H, dt) - lo
        assert k in steps
        if steps.size == 1:
            monotone += 1
            assert k == np.flatnonzero(ok)[0]
    assert monotone >= 1


def test_gap_variant_refinement():
    """q = 2, 3 of Sec. 4.7.  A run of consecutive floats has q-gaps of q ulps, which keeps the
    rounding of m(H D) finer than the spacing of the q-pairs, so growth there is by one float
    (seen on random arrays started at Hbar); the pins hold as for q = 1, and q = 1 of the gap
    variant equals plain Direct."""
    rng = np.random.default_rng(41)
    found = 0
    for q in (2, 3):
        for form in (oracle.FORM_SUB, oracle.FORM_FMA):
            for _ in range(3000):
                x0 = 0.0 if form == oracle.FORM_SUB else rng.uniform(-100, 100)
                X = (x0 + np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 5.0, 15))])).astype(np.float32)
                if oracle.compute_hr_gap(X, q, form, oracle.HSTART_HBAR).n_updates:
                    _check_refined(X, q, form, oracle.HSTART_HBAR)
                    found += 1
    assert found >= 20
    for form in (oracle.FORM_SUB, oracle.FORM_FMA):
        for X in _growth_cases(np.float32, form, 1, 10, seed=50 + form):
            a = oracle.compute_hr(X, form, refine=True)
            b = oracle.compute_hr_gap(X, 1, form, refine=True)
            assert (a.H, a.W, a.R, a.jmin, a.n_refine, a.H_lo) == (b.H, b.W, b.R, b.jmin, b.n_refine, b.H_lo)


def test_no_growth_means_no_change():
    for dt in (np.float32, np.float64):
        for n in (16, 4096):
            X = W.sweep_array(n, dt)
            for form in (oracle.FORM_SUB, oracle.FORM_FMA):
                g = oracle.build_direct(X, form)
                r = oracle.build_direct(X, form, refine=True)
                assert g.n_updates == 0 and g.H_bad == 0.0
                assert (r.H, r.W, r.R, r.jmin, r.n_refine) == (g.H, g.W, g.R, g.jmin, 0)
                assert np.array_equal(r.K, g.K)


def test_paper_arrays_grow_by_one_float():
    """The arrays of the table of H updates (Sec. 6.6; gaps U[1, 5], H started at Hbar): where
    H grows it grows by one float, so the refinement has nothing to bisect, which is the
    paper's reason for leaving it out."""
    rng = np.random.default_rng(11)
    grown = 0
    for _ in range(3000):
        X = np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 5.0, 15))]).astype(np.float32)
        g = oracle.compute_hr(X, hstart=oracle.HSTART_HBAR)
        if g.n_updates:
            grown += 1
            r = oracle.compute_hr(X, hstart=oracle.HSTART_HBAR, refine=True)
            assert np.nextafter(np.float32(g.H_bad), np.float32(np.inf)) == np.float32(g.H)
            assert r.H == g.H and r.n_refine == 0
    assert grown > 0


def test_refine_rejects_bad_intervals():
    X = _growth_cases(np.float32, oracle.FORM_SUB, 1, 1, seed=60)[0]
    g = oracle.compute_hr(X)
    n = X.size - 1
    assert oracle.refine_h(X, 1, 0, g.H_bad, g.H_grown)[0] == oracle.OK
    assert oracle.refine_h(X, 1, 0, g.H_grown, g.H_bad)[0] == oracle.ERR_ARG    # lo >= hi
    assert oracle.refine_h(X, 1, 0, g.H_grown, 2 * g.H_grown)[0] == oracle.ERR_ARG  # lo feasible
    assert oracle.refine_h(X, 1, 0, g.H_bad / 4, g.H_bad)[0] == oracle.ERR_ARG  # hi infeasible
    assert oracle.refine_h(X, 0, 0, g.H_bad, g.H_grown)[0] == oracle.ERR_ARG
    assert oracle.refine_h(X, n + 1, 0, g.H_bad, g.H_grown)[0] == oracle.ERR_ARG
