"""GPU parity of the scalar-problem device API and of the fused uses of Sec. 2
(histogram per interval, piecewise-linear interpolation) against the oracle.

ds_view_search (a kernel built on ds_device.h alone) must equal the oracle's
search element by element.  ds_histogram must equal the oracle's bincount of
its search bit for bit, for the LDS-private bins (small N) and the global
counters (large N), accumulating over calls; at N = 2^21 with 2^26 f64 queries
the whole histogram is compared.  ds_interp_linear must equal the oracle's
same-precision evaluation of the documented formula bit for bit (both are IEEE
operations in the same order without contraction).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import apps

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SIZES = [16, 256, 4096, 65536, 1 << 20]


@pytest.fixture(scope="module")
def ds():
    import paper_1506_08620_amd as mod

    return mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _assert_same(got, ref, z=None):
    if not np.array_equal(got, ref, equal_nan=np.issubdtype(np.asarray(ref).dtype, np.floating)):
        bad = np.flatnonzero(~((got == ref) | (np.isnan(got) & np.isnan(ref)))) if np.issubdtype(
            np.asarray(ref).dtype, np.floating) else np.flatnonzero(got != ref)
        raise AssertionError(f"{bad.size} of {ref.size} differ; first {bad[:4]}: got {got[bad[:4]]} "
                             f"want {ref[bad[:4]]}" + (f" z={z[bad[:4]]}" if z is not None else ""))


def _queries(X, rng, m=200_000):
    dt = X.dtype
    return np.concatenate([W.uniform_queries(X[0], X[-1], m, dt, rng), X, W.prev_float(X, dt),
                           np.nextafter(X, dt.type(np.inf)),
                           np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, -1.0, 1e30], dt)]).astype(dt)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_view_search_equals_oracle(ds, dtype):
    rng = np.random.default_rng(1)
    for n in SIZES:
        X = W.sweep_array(n, dtype)
        z = _queries(X, rng)
        ref = oracle.search(X, z)
        for form in ("sub", "fma"):
            idx = ds.build(_dev(X), form=form)
            v = idx.view()
            assert v.N == n and v.dtype == (0 if dtype == np.float32 else 1)
            _assert_same(ds.view_search(v, _dev(z)).cpu().numpy(), ref, z)
            idx.destroy()
    idx = ds.build(_dev(W.sweep_array(16, dtype)), method="leadbit")
    with pytest.raises(ds.DsError) as e:
        idx.view()
    assert e.value.status == ds.ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_histogram_equals_oracle(ds, dtype):
    rng = np.random.default_rng(2)
    for n in SIZES:
        X = W.sweep_array(n, dtype)
        z = _queries(X, rng)
        ref = apps.histogram(X, z)
        for form in ("sub", "fma"):
            idx = ds.build(_dev(X), form=form)
            h = idx.histogram(_dev(z)).cpu().numpy()
            _assert_same(h, ref)
            # accumulates; and an unaligned query pointer takes the scalar path
            counts = torch.zeros(n + 2, dtype=torch.int64, device=DEV)
            idx.histogram(_dev(z), counts)
            zd = _dev(np.concatenate([[X[0]], z]).astype(dtype))[1:]
            idx.histogram(zd, counts)
            _assert_same(counts.cpu().numpy(), 2 * ref)
            idx.destroy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_interp_linear_equals_oracle(ds, dtype):
    rng = np.random.default_rng(3)
    for n in SIZES:
        X = W.sweep_array(n, dtype)
        Y = np.cumsum(rng.normal(0, 1, n + 1)).astype(dtype)
        z = _queries(X, rng)
        ref = apps.interp_linear(X, Y, z)
        for form in ("sub", "fma"):
            idx = ds.build(_dev(X), form=form)
            y = idx.interp_linear(_dev(Y), _dev(z)).cpu().numpy()
            _assert_same(y, ref, z)
            zd = _dev(np.concatenate([[X[0]], z]).astype(dtype))[1:]
            _assert_same(idx.interp_linear(_dev(Y), zd).cpu().numpy(), ref, z)
            idx.destroy()


def test_apps_reject_other_methods(ds):
    X = W.sweep_array(64, np.float32)
    idx = ds.build(_dev(X), method="eytzinger")
    z = _dev(X)
    with pytest.raises(ds.DsError) as e:
        idx.histogram(z)
    assert e.value.status == ds.ERR_UNSUPPORTED
    with pytest.raises(ds.DsError) as e:
        idx.interp_linear(_dev(X), z)
    assert e.value.status == ds.ERR_UNSUPPORTED


def test_full_size_histogram_and_interp_f64(ds):
    """N = 2^21 (NIBBLE layout through L2, global counters), 2^26 queries."""
    X = W.sweep_array(1 << 21, np.float64)
    M = 1 << 26
    z = W.sweep_queries_torch(M, np.float64, DEV)
    idx = ds.build(_dev(X))
    assert idx.info()["staged"] == 6
    h = idx.histogram(z).cpu().numpy()
    zh = z.cpu().numpy()
    _assert_same(h, apps.histogram(X, zh))
    Y = np.cumsum(np.random.default_rng(4).normal(0, 1, X.size))
    y = idx.interp_linear(_dev(Y), z)
    pos = np.random.default_rng(5).integers(0, M, 1 << 18)
    _assert_same(y[torch.from_numpy(pos).to(DEV)].cpu().numpy(), apps.interp_linear(X, Y, zh[pos]), zh[pos])
