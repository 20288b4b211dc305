"""GPU parity of the gap-q variant of Sec. 4.7 (method "direct_gap") against the oracle.

The build's H, W, R, jmin, number of H updates and table K (eq. (kgeneral)) are
compared bit for bit with the oracle's gap-q ComputeHR and table; the search is
compared element by element with the oracle's classic binary search on every
layout it runs on (padded X and K in LDS, or through L2), in both forms of the
grid map, for q = 1..16.  At the full sweep size (N = 2^21, 2^26 queries) the
outputs are sampled against the oracle and the defining invariant is checked
for every query on the device.
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


def _queries(X, rng, m=100_000):
    dt = X.dtype
    return np.concatenate([W.uniform_queries(X[0], X[-1], m, dt, rng), X, W.prev_float(X, dt),
                           np.nextafter(X, dt.type(np.inf)),
                           np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, -1.0, 1e30], dt)]).astype(dt)


def _check_tables(idx, X, q, form):
    t = oracle.build_direct_gap(X, q, FORMS[form])
    assert t.status == oracle.OK
    inf = idx.info()
    assert inf["method_name"] == "direct_gap" and inf["gap_q"] == q
    assert inf["H"] == t.H and inf["W"] == t.W and inf["R"] == t.R and inf["jmin"] == t.jmin
    assert inf["n_h_updates"] == t.n_updates
    assert np.array_equal(idx.table().cpu().numpy(), t.K)
    return inf


def _stages(inf):
    """The layouts a handle can be searched through: PLAIN in LDS (when it fits) and through
    L2, and GAPCODE in LDS (q <= 3, when it fits)."""
    st = [1, 2] if inf["staged"] == 1 else [2]
    if inf["gapcode_bytes"] and inf["gapcode_bytes"] <= 160 * 1024 - 64:
        st.append(8)
    return tuple(st)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [16, 256, 4096, 65536])
def test_gap_tables_and_indices(ds, dtype, n):
    rng = np.random.default_rng(n)
    X = W.sweep_array(n, dtype)
    z = _queries(X, rng)
    ref = oracle.search(X, z)
    for form in ("sub", "fma"):
        for q in (1, 2, 3, 4, 8, 16):
            if q > n:
                continue
            idx = ds.build(_dev(X), method="direct_gap", gap_q=q, form=form)
            inf = _check_tables(idx, X, q, form)
            for stage in _stages(inf):
                idx.set_tune(stage=stage)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            idx.destroy()


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_gapcode_ties_on_twin_keys(ds, form):
    """GAPCODE (stage 8) where the codes tie: "twin" arrays, pairs of consecutive floats about
    one unit apart, which a q = 2 grid puts in one cell each (so the pair's position codes are
    equal or adjacent and X decides); q = 3 (2-bit counts) and q = 4, 9 (4-bit counts) too.  Every key, the floats next to every key and
    out-of-domain values, against the oracle."""
    rng = np.random.default_rng(44)
    for a in range(12):
        dt = np.dtype(np.float32 if a % 2 else np.float64)
        n_pairs = int(rng.integers(3, 20_000))
        base = (np.cumsum(rng.uniform(0.8, 1.2, n_pairs)) + rng.uniform(-500, 500)).astype(dt)
        X = np.unique(np.concatenate([base, np.nextafter(base, dt.type(np.inf))]))
        for q in (2, 3, 4, 9):  # 2-bit and 4-bit cell counts
            if oracle.build_direct_gap(X, q, FORMS[form]).status != oracle.OK:
                continue
            z = _queries(X, rng, m=20_000)
            ref = oracle.search(X, z)
            idx = ds.build(_dev(X), method="direct_gap", gap_q=q, form=form)
            _check_tables(idx, X, q, form)
            idx.set_tune(stage=8)
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            idx.destroy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("q", [2, 4, 15])
def test_gapcode_keeps_gap_q_on_chip_at_65536(ds, dtype, q):
    """N = 65536: the PLAIN table and X do not fit LDS but GAPCODE does, and the automatic
    launch uses it; 2^22 sweep queries equal the oracle."""
    X = W.sweep_array(65536, dtype)
    idx = ds.build(_dev(X), method="direct_gap", gap_q=q)
    inf = idx.info()
    assert inf["staged"] == 8 and 0 < inf["gapcode_bytes"] <= 160 * 1024
    z = W.sweep_queries(1 << 22, dtype)
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z), z)


def test_gap_tiny_arrays_and_unaligned(ds):
    """N from q to 40 with random gaps, every q, both forms; unaligned query pointers take the
    scalar path."""
    rng = np.random.default_rng(3)
    for dtype in (np.float32, np.float64):
        for n in (1, 2, 3, 5, 17, 40):
            X = W.gap_array(n, dtype, rng, lo=0.1, hi=2.0, x0=rng.uniform(-3, 3))
            z = _queries(X, rng, m=5000)
            ref = oracle.search(X, z)
            for q in range(1, min(n, 16) + 1):
                for form in ("sub", "fma"):
                    idx = ds.build(_dev(X), method="direct_gap", gap_q=q, form=form)
                    _check_tables(idx, X, q, form)
                    zd = _dev(np.concatenate([[X[0]], z]).astype(dtype))[1:]  # 1-element offset
                    _assert_same(ds.search(idx, zd).cpu().numpy(), ref, z)
                    idx.destroy()


def test_gap_launch_shapes(ds):
    X = W.sweep_array(4096, np.float32)
    z = _queries(X, np.random.default_rng(1), m=300_001)
    ref = oracle.search(X, z)
    idx = ds.build(_dev(X), method="direct_gap", gap_q=3)
    for stage in (1, 2, 8):
        for block in (64, 256, 1024):
            for unroll in (1, 2, 4):
                idx.set_tune(block=block, unroll=unroll, stage=stage, grid=0 if block != 64 else 7)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref)
    with pytest.raises(ds.DsError):
        idx.set_tune(stage=3)


def test_gap_relaxed_feasibility(ds):
    """Two keys one float apart at 1e-10 in [-0.5, 0.5] defeat plain Direct (their rounded
    offsets from X_0 coincide); q = 2 builds and is exact, and the automatic q picks 2."""
    rng = np.random.default_rng(4)
    for dt in (np.float32, np.float64):
        base = (np.cumsum(rng.uniform(0.5, 1.5, 1000)) / 1000.0 - 0.5).astype(dt)
        base = base[np.abs(base) > 1e-3]
        a = dt(1e-10)
        X = np.sort(np.concatenate([[dt(-0.5)], base, [a, np.nextafter(a, dt(np.inf))]])).astype(dt)
        with pytest.raises(ds.DsError) as e:
            ds.build(_dev(X))
        assert e.value.status == ds.ERR_INFEASIBLE
        z = _queries(X, rng)
        ref = oracle.search(X, z)
        for q in (2, 0):
            idx = ds.build(_dev(X), method="direct_gap", gap_q=q)
            inf = _check_tables(idx, X, 2, "sub")
            for stage in _stages(inf):
                idx.set_tune(stage=stage)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)


def test_gap_q_from_memory_budget(ds):
    """gap_q = 0: the smallest q whose grid is feasible and whose table (4 bytes per cell)
    fits table_cap_bytes, found by the same loop over the oracle."""
    X = W.sweep_array(65536, np.float64)
    z = _queries(X, np.random.default_rng(2))
    ref = oracle.search(X, z)
    for cap in (600_000, 300_000, 100_000, 40_000):
        want = None
        for q in range(1, 17):
            t = oracle.compute_hr_gap(X, q)
            if t.status == oracle.OK and (t.R - t.jmin + 1) * 4 <= cap:
                want = q
                break
        assert want is not None
        idx = ds.build(_dev(X), method="direct_gap", gap_q=0, table_cap_bytes=cap)
        inf = _check_tables(idx, X, want, "sub")
        assert inf["table_bytes"] <= cap
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref)
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(X), method="direct_gap", gap_q=0, table_cap_bytes=1000)
    assert e.value.status == ds.ERR_TABLE_CAP


def test_gap_errors_and_fallback(ds):
    X = W.sweep_array(16, np.float32)
    for q in (17, -1):
        with pytest.raises(ds.DsError) as e:
            ds.build(_dev(X), method="direct_gap", gap_q=q)
        assert e.value.status == ds.ERR_ARG
    X3 = X[:4].copy()  # N = 3
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(X3), method="direct_gap", gap_q=4)
    assert e.value.status == ds.ERR_ARG
    # three keys one float apart at 1e-10 in [-0.5, 0.5] defeat q = 2 (their rounded offsets
    # from X_0 coincide); the fallback builds the leading-bit search instead
    rng = np.random.default_rng(8)
    base = (np.cumsum(rng.uniform(0.5, 1.5, 1000)) / 1000.0 - 0.5).astype(np.float32)
    base = base[np.abs(base) > 1e-3]
    a = np.float32(1e-10)
    b = np.nextafter(a, np.float32(1))
    c = np.nextafter(b, np.float32(1))
    Xb = np.sort(np.concatenate([[np.float32(-0.5)], base, [a, b, c]])).astype(np.float32)
    assert oracle.compute_hr_gap(Xb, 2).status == oracle.ERR_INFEASIBLE
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(Xb), method="direct_gap", gap_q=2)
    assert e.value.status == ds.ERR_INFEASIBLE
    idx = ds.build(_dev(Xb), method="direct_gap", gap_q=2, fallback="bsearch")
    assert idx.info()["method_name"] == "leadbit"
    z = _queries(Xb, rng, m=10_000)
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(Xb, z))
    idx = ds.build(_dev(Xb), method="direct_gap", gap_q=3)
    _check_tables(idx, Xb, 3, "sub")
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(Xb, z))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_gap_full_size_sampled(ds, dtype):
    """N = 2^21, 2^26 queries (the sweep's largest case) through L2, q = 2 and 4."""
    X = W.sweep_array(1 << 21, dtype)
    M = 1 << 26
    xd = _dev(X)
    z = W.sweep_queries_torch(M, dtype, DEV)
    for q in (2, 4):
        idx = ds.build(xd, method="direct_gap", gap_q=q)
        inf = idx.info()
        t = oracle.compute_hr_gap(X, q)
        assert (inf["H"], inf["R"], inf["n_h_updates"]) == (t.H, t.R, t.n_updates)
        out = ds.search(idx, z)
        i = out.long()
        assert int(i.min()) >= 0 and int(i.max()) <= X.size - 2
        assert bool(torch.all(xd[i] <= z)) and bool(torch.all(z < xd[i + 1]))
        pos = torch.from_numpy(np.random.default_rng(q).integers(0, M, 1 << 18)).to(DEV)
        zs = z[pos].cpu().numpy()
        _assert_same(out[pos].cpu().numpy(), oracle.search(X, zs), zs)
        idx.destroy()
