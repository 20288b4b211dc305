"""GPU parity of the H refinement (the bisection of [last infeasible H, grown H]
proposed at the end of Sec. 4.4.3; ds_build_opts.refine_h) against the oracle.

Arrays at the feasibility limit (smallest gap about one ulp of the largest key,
workloads.near_limit_array), where ComputeHR grows H by up to 23 doublings of its
step, are built with and without the refinement; H, W, R, jmin, the number of H
updates and of bisection midpoints, and the whole table K must equal the oracle's
bit for bit, and the search on every layout must equal the oracle's search
element by element.  Filler keys take N from 16 to about 2^18 (several tiles of
the verify and fill kernels, ragged tails).  The gap variant (Sec. 4.7) is checked
on random arrays started at Hbar, and arrays on which H never grows must come out
unchanged.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
FORMS = {"sub": oracle.FORM_SUB, "fma": oracle.FORM_FMA}


@pytest.fixture(scope="module")
def ds():
    import paper_1506_08620_amd as mod

    return mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _assert_same(got, ref, z=None):
    if not np.array_equal(got, ref):
        bad = np.flatnonzero(got != ref)
        raise AssertionError(f"{bad.size} of {ref.size} differ; first {bad[:4]}: got {got[bad[:4]]} "
                             f"want {ref[bad[:4]]}" + (f" z={z[bad[:4]]}" if z is not None else ""))


def _queries(X, rng, m=200_000):
    dt = X.dtype
    return np.concatenate([W.uniform_queries(X[0], X[-1], m, dt, rng), X, W.prev_float(X, dt),
                           np.nextafter(X, dt.type(np.inf)),
                           np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, -1.0, 1e30], dt)]).astype(dt)


def _growth_cases(form, n_fill, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(400):
        X = W.near_limit_array(np.float32, rng, n_fill=n_fill)
        t = oracle.compute_hr(X, form)
        if t.status == oracle.OK and t.n_updates >= 2 and t.R < (1 << 26):  # tables up to 256 MB
            out.append(X)
            if len(out) == count:
                break
    assert len(out) == count
    return out


def _stages(inf):
    st = [2]
    if inf["staged"] == 1:
        st.append(1)
    if inf["rankcode_bytes"] and inf["rankcode_bytes"] <= 160 * 1024 - 64:
        st.append(3)
    for key, stage in (("pairs_bytes", 4), ("rankcode_bytes", 5), ("nibble_bytes", 6)):
        if inf[key]:
            st.append(stage)
    if inf["nibble_bytes"] and inf["nibble_bytes"] <= 160 * 1024:
        st.append(7)
    return st


def _check_info(inf, t, refined):
    assert inf["H"] == t.H and inf["W"] == t.W and inf["R"] == t.R and inf["jmin"] == t.jmin
    assert inf["n_h_updates"] == t.n_updates
    assert inf["n_h_refine"] == (t.n_refine if refined else 0)


@pytest.mark.parametrize("form", ["sub", "fma"])
@pytest.mark.parametrize("n_fill", [0, 300, 20_000, 250_000])
def test_refined_build_equals_oracle(ds, form, n_fill):
    rng = np.random.default_rng(n_fill)
    for X in _growth_cases(FORMS[form], n_fill, 2, seed=100 + n_fill + FORMS[form]):
        grown = oracle.build_direct(X, FORMS[form])
        ref = oracle.build_direct(X, FORMS[form], refine=True)
        assert ref.status == oracle.OK and ref.n_refine > 0 and ref.R <= grown.R
        xd = _dev(X)
        idx = ds.build(xd, form=form)
        _check_info(idx.info(), grown, False)
        idx.destroy()
        layouts = ("rankcode", "pairs", "nibble") if X.size < 100_000 else ("nibble",)
        idx = ds.build(xd, form=form, refine_h=True, layouts=layouts)
        inf = idx.info()
        _check_info(inf, ref, True)
        assert np.array_equal(idx.table().cpu().numpy(), ref.K)
        z = _queries(X, rng)
        want = oracle.search(X, z)
        for stage in _stages(inf):
            idx.set_tune(stage=stage)
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), want, z)
        idx.destroy()


def test_refined_build_with_an_offset_x0_in_the_fma_form(ds):
    rng = np.random.default_rng(5)
    found = 0
    for _ in range(20_000):
        X = W.near_limit_array(np.float32, rng, offset=True)
        t = oracle.compute_hr(X, oracle.FORM_FMA)
        if t.status != oracle.OK or t.n_updates < 2:
            continue
        ref = oracle.build_direct(X, oracle.FORM_FMA, refine=True)
        idx = ds.build(_dev(X), form="fma", refine_h=True)
        _check_info(idx.info(), ref, True)
        assert np.array_equal(idx.table().cpu().numpy(), ref.K)
        z = _queries(X, rng, m=20_000)
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z), z)
        idx.destroy()
        found += 1
        if found == 3:
            break
    assert found >= 1


def test_refined_gap_variant(ds):
    """q = 2, 3 on random arrays (gaps U[1, 5], H started at Hbar) where H grows."""
    rng = np.random.default_rng(41)
    found = 0
    for q in (2, 3):
        for form in ("sub", "fma"):
            hits = 0
            for _ in range(3000):
                x0 = 0.0 if form == "sub" else rng.uniform(-100, 100)
                X = (x0 + np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 5.0, 15))])).astype(np.float32)
                t = oracle.build_direct_gap(X, q, FORMS[form], oracle.HSTART_HBAR, refine=True)
                if not t.n_updates:
                    continue
                idx = ds.build(_dev(X), method="direct_gap", gap_q=q, form=form, hstart="hbar", refine_h=True)
                inf = idx.info()
                _check_info(inf, t, True)
                assert inf["gap_q"] == q
                assert np.array_equal(idx.table().cpu().numpy(), t.K)
                z = _queries(X, rng, m=5000)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z), z)
                idx.destroy()
                hits += 1
                if hits == 3:
                    break
            found += hits
    assert found >= 6


def test_refine_leaves_arrays_without_growth_unchanged(ds):
    for dt in (np.float32, np.float64):
        for n in (16, 4096, 1 << 20):
            X = W.sweep_array(n, dt)
            xd = _dev(X)
            for form in ("sub", "fma"):
                a = ds.build(xd, form=form).info()
                b = ds.build(xd, form=form, refine_h=True).info()
                assert a["n_h_updates"] == 0 and b["n_h_refine"] == 0
                assert (a["H"], a["W"], a["R"], a["jmin"]) == (b["H"], b["W"], b["R"], b["jmin"])


def test_refine_h_value_is_checked(ds):
    import ctypes

    X = _dev(W.sweep_array(16, np.float32))
    opts = ds.BuildOpts()
    opts.refine_h = 2
    h = ctypes.c_void_p()
    st = ds._lib.ds_build(X.data_ptr(), 16, 0, ctypes.byref(opts), None, ctypes.byref(h))
    assert st == ds.ERR_ARG
