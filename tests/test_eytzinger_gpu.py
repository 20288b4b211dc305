"""GPU parity of the Eytzinger binary search (Sec. 3.4, method "eytzinger") against the oracle.

Every result is compared element by element with the oracle's classic binary
search, with the top levels of the tree in LDS and with every level through
L2, over the N sweep, tiny arrays, unaligned pointers and every launch shape;
at N = 2^21 with 2^26 queries outputs are sampled and the defining invariant
is checked for every query on the device.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


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


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [16, 256, 4096, 65536, 1 << 20])
def test_eytzinger_sweep_both_stages(ds, dtype, n):
    rng = np.random.default_rng(n)
    X = W.sweep_array(n, dtype)
    z = _queries(X, rng, m=200_000)
    ref = oracle.search(X, z)
    idx = ds.build(_dev(X), method="eytzinger")
    inf = idx.info()
    assert inf["method_name"] == "eytzinger" and inf["staged"] == 1
    L = oracle.eytzinger_levels(n)
    assert inf["x_bytes"] == (1 << L) * np.dtype(dtype).itemsize
    for stage in (1, 2):
        idx.set_tune(stage=stage)
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
    with pytest.raises(ds.DsError):
        idx.set_tune(stage=3)


def test_eytzinger_tiny_and_unaligned(ds):
    rng = np.random.default_rng(5)
    for dtype in (np.float32, np.float64):
        for n in (1, 2, 3, 6, 7, 8, 14, 15, 16, 31, 33, 100):
            X = W.gap_array(n, dtype, rng, lo=0.1, hi=2.0, x0=rng.uniform(-3, 3))
            z = _queries(X, rng, m=3000)
            ref = oracle.search(X, z)
            idx = ds.build(_dev(X), method="eytzinger")
            for stage in (1, 2):
                idx.set_tune(stage=stage)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
                zd = _dev(np.concatenate([[X[0]], z]).astype(dtype))[1:]
                _assert_same(ds.search(idx, zd).cpu().numpy(), ref, z)


def test_eytzinger_launch_shapes(ds):
    X = W.sweep_array(65536, np.float64)
    z = _queries(X, np.random.default_rng(1), m=300_001)
    ref = oracle.search(X, z)
    idx = ds.build(_dev(X), method="eytzinger")
    for stage in (1, 2):
        for block in (64, 256, 1024):
            for unroll in (1, 2, 4):
                idx.set_tune(block=block, unroll=unroll, stage=stage, grid=0 if block != 64 else 5)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref)
    best = idx.autotune(_dev(z))
    assert best["stage"] in (1, 2)
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_eytzinger_full_size_sampled(ds, dtype):
    X = W.sweep_array(1 << 21, dtype)
    M = 1 << 26
    xd = _dev(X)
    z = W.sweep_queries_torch(M, dtype, DEV)
    idx = ds.build(xd, method="eytzinger")
    out = ds.search(idx, z)
    i = out.long()
    assert int(i.min()) >= 0 and int(i.max()) <= X.size - 2
    assert bool(torch.all(xd[i] <= z)) and bool(torch.all(z < xd[i + 1]))
    pos = torch.from_numpy(np.random.default_rng(7).integers(0, M, 1 << 18)).to(DEV)
    zs = z[pos].cpu().numpy()
    _assert_same(out[pos].cpu().numpy(), oracle.search(X, zs), zs)
