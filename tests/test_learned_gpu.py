"""GPU checks of the learned CDF method: the training kernels' gradients and the
search-time router against the fp64 reference, monotone routing, and exact
indices against the oracle on clustered arrays (where Direct is infeasible)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import mlp

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ds():
    import paper_1506_08620_amd as mod

    return mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _params(rng):
    p = np.empty(mlp.N_PARAMS)
    w1 = rng.uniform(2, 6, 32)
    c = rng.uniform(0.1, 0.9, 32)
    p[0:32] = w1
    p[32:64] = 0.5 - w1 * c
    W2 = rng.uniform(0, 2.0 / 32, (32, 32))
    p[64:1088] = W2.reshape(-1)
    p[1088:1120] = 0.5 - 0.5 * W2.sum(1) + rng.uniform(-0.1, 0.1, 32)
    p[1120:1152] = rng.uniform(0, 1.0 / 16, 32)
    p[1152] = rng.uniform(-0.1, 0.1)
    return p.astype(np.float32)


def _assert_same(got, ref, z=None):
    if not np.array_equal(got, ref):
        bad = np.flatnonzero(got != ref)
        raise AssertionError(f"{bad.size} of {ref.size} differ; first {bad[:4]}: got {got[bad[:4]]} "
                             f"want {ref[bad[:4]]}" + (f" z={z[bad[:4]]}" if z is not None else ""))


def test_training_gradients_match_fp64_reference(ds):
    """GPU fp32 gradients vs CPU fp64 at fixed weights on a fixed batch: relative L2 <= 1e-3 per tensor."""
    rng = np.random.default_rng(5)
    for trial in range(3):
        p = _params(rng)
        u = rng.uniform(0, 1, 3000).astype(np.float32)
        t = np.sort(rng.uniform(0, 1, 3000)).astype(np.float32)
        loss_g, g = ds.learned_grad(_dev(p), _dev(u), _dev(t))
        loss_c, gc = mlp.grad(p.astype(np.float64), u.astype(np.float64), t.astype(np.float64))
        g = g.cpu().numpy().astype(np.float64)
        assert abs(loss_g - loss_c) <= 1e-4 * max(loss_c, 1e-12)
        for name, a, b in (("W1", 0, 32), ("b1", 32, 64), ("W2", 64, 1088), ("b2", 1088, 1120),
                           ("W3", 1120, 1152), ("b3", 1152, 1153)):
            ref = gc[a:b]
            err = np.linalg.norm(g[a:b] - ref) / max(np.linalg.norm(ref), 1e-12)
            assert err <= 1e-3, (trial, name, err)


def test_search_router_matches_reference_and_is_monotone(ds):
    rng = np.random.default_rng(6)
    p = _params(rng)
    u = np.sort(np.concatenate([rng.uniform(0, 1, 200_000), np.linspace(0, 1, 4097)])).astype(np.float32)
    y = ds.learned_forward(_dev(p), _dev(u)).cpu().numpy()
    yc, _ = mlp.forward(p.astype(np.float64), u.astype(np.float64))
    # 32-term fp32 dot products of values in [0, 1]: errors of a few 1e-7, bounded well below 1e-4
    assert np.max(np.abs(y - yc)) < 1e-4
    assert np.all(np.diff(y) >= 0)  # exact: non-negative weights, monotone rounding
    # FP16 inputs to the 32x32 layer: relative rounding 2^-11 of h1 and W2, so |y - y_ref| of a
    # few 1e-3 at most for these weights; still exactly monotone
    y16 = ds.learned_forward(_dev(p), _dev(u), fp16_router=True).cpu().numpy()
    assert np.max(np.abs(y16 - yc)) < 5e-3
    assert np.all(np.diff(y16) >= 0)


def _clustered(n, dt, seed):
    rng = np.random.default_rng(seed)
    x = np.unique(np.exp(rng.normal(0, 2, n * 2)).astype(dt))[: n + 1]
    return x


def _queries(X, m, rng):
    dt = X.dtype
    zu = W.uniform_queries(X[0], X[-1], m, dt, rng)
    k = rng.integers(0, X.size, m)
    zc = (X[k].astype(np.float64) * (1 + rng.uniform(-1e-6, 1e-6, m))).astype(dt)
    zc = np.clip(zc, X[0], W.prev_float(X[-1], dt))
    extra = [X, W.prev_float(X, dt), np.nextafter(X, dt.type(np.inf)),
             np.array([np.nan, np.inf, -np.inf, 0.0, -1.0, 1e30], dt)]
    return np.concatenate([zu, zc, *extra]).astype(dt)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_learned_exact_on_clustered_arrays(ds, dt):
    rng = np.random.default_rng(7)
    for n, segs in ((50, 16), (3000, 256), (40_000, 4096)):
        X = _clustered(n, dt, n)
        z = _queries(X, 100_000, rng)
        ref = oracle.search(X, z)
        # trained router (compiled step table; evaluated per query with FP16 / FP32 inputs), no network
        for epochs, router in ((20, "table"), (20, "fp16"), (20, "fp32"), (-1, "table")):
            idx = ds.build(_dev(X), method="learned", learn_epochs=epochs, learn_segments=segs, seed=3,
                           learn_router=router)
            inf = idx.info()
            assert inf["method_name"] == "learned"
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            _, fb = idx.learned_model()
            assert fb == 0
            torch.cuda.synchronize()
            assert idx.info()["fallback_count"] == 0
            table = router == "table" and epochs > 0
            # fits (32 bytes each); the compiled router adds its steps (4 bytes per segment) and a grid of
            # as many 4-byte cells as segments
            assert inf["model_bytes"] == 1153 * 4 + segs * (40 if table else 32)


def test_compiled_router_is_the_fp32_network(ds):
    """The step table routes every f32 feature exactly as the FP32 network evaluated on it does:
    on random features, on a grid, and on both sides of every step of the network, each found by
    bisection over f32 bit patterns with the evaluated network (mode 1), for the search's routing
    (mode 0, grid then steps) and the build's (mode 2, the whole table)."""
    rng = np.random.default_rng(11)
    one = int(np.float32(1.0).view(np.uint32))
    for dt, n, segs in ((np.float64, 200_000, 2048), (np.float32, 30_000, 512), (np.float64, 5_000, 4096)):
        X = _clustered(n, dt, 17)
        idx = ds.build(_dev(X), method="learned", learn_epochs=20, learn_segments=segs, seed=9)
        u = np.concatenate([rng.uniform(0, 1, 1 << 20), np.linspace(0, 1, 65537), [0.0, 1.0]]).astype(np.float32)
        ud = _dev(u)
        net = idx.learned_route(ud, 1).cpu().numpy()
        assert np.all(net >= 0) and np.all(net < segs)
        for mode in (0, 2):
            assert np.array_equal(idx.learned_route(ud, mode).cpu().numpy(), net), (dt, n, mode)
        # brackets where the network's segment changes on a grid of bit patterns, then bisection
        bits = np.unique(np.linspace(0, one, 1 << 20).astype(np.int64))
        sg = idx.learned_route(_dev(bits.astype(np.uint32).view(np.float32)), 1).cpu().numpy()
        assert np.all(np.diff(sg) >= 0)  # the network's segment is non-decreasing in u
        ch = np.flatnonzero(np.diff(sg))
        lo, hi = bits[ch], bits[ch + 1]
        s_lo = sg[ch]
        while np.any(hi - lo > 1):
            mid = lo + (hi - lo) // 2
            sm = idx.learned_route(_dev(mid.astype(np.uint32).view(np.float32)), 1).cpu().numpy()
            same = sm == s_lo
            lo = np.where(same, mid, lo)
            hi = np.where(same, hi, mid)
        edge = np.concatenate([lo, hi]).astype(np.uint32).view(np.float32)
        ed = _dev(edge)
        ref = idx.learned_route(ed, 1).cpu().numpy()
        assert np.all(ref[: lo.size] < ref[lo.size:])  # a step between each pair of neighbouring floats
        for mode in (0, 2):
            assert np.array_equal(idx.learned_route(ed, mode).cpu().numpy(), ref), (dt, n, mode)
        idx.destroy()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_learned_wide_windows_and_array_ends(ds, dt):
    """Few segments over many keys give windows of thousands of keys (the search narrows them by
    bisection on the samples of X's 64-byte blocks before reading one block); sizes around a
    block multiple put the last window at the padded end of X."""
    rng = np.random.default_rng(17)
    for n, segs in ((200_000, 4), (200_000, 16), (8 * 1024 - 1, 64), (8 * 1024, 64), (16 * 1024 + 1, 64)):
        X = _clustered(n, dt, n)
        z = _queries(X, 50_000, rng)
        ref = oracle.search(X, z)
        for epochs in (5, -1):
            idx = ds.build(_dev(X), method="learned", learn_epochs=epochs, learn_segments=segs, seed=5)
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            _, fb = idx.learned_model()
            assert fb == 0
            idx.destroy()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_learned_segment_counts_off_four(ds, dt):
    """Segment counts that are not multiples of 4 (1, 3, 5, 37, 1023) place the compiled router's
    grid, after the step table, off a 16-byte boundary in LDS: exact results without fallback,
    trained and without network."""
    rng = np.random.default_rng(19)
    X = _clustered(20_000, dt, 20_000)
    z = _queries(X, 40_000, rng)
    ref = oracle.search(X, z)
    for segs in (1, 3, 5, 37, 1023):
        for epochs in (5, -1):
            idx = ds.build(_dev(X), method="learned", learn_epochs=epochs, learn_segments=segs, seed=8)
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            _, fb = idx.learned_model()
            assert fb == 0
            idx.destroy()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_learned_tiny_arrays(ds, dt):
    """N from 1 to 33 (one block of X or a few; the padded tail of X and of the samples is read)."""
    rng = np.random.default_rng(23)
    for n in (1, 2, 3, 7, 8, 9, 15, 16, 17, 33):
        X = W.gap_array(n, dt, rng, lo=0.1, hi=3.0, x0=rng.uniform(-5, 5))
        z = _queries(X, 2000, rng)
        ref = oracle.search(X, z)
        for epochs in (3, -1):
            idx = ds.build(_dev(X), method="learned", learn_epochs=epochs, learn_segments=16, seed=2)
            _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
            _, fb = idx.learned_model()
            assert fb == 0
            idx.destroy()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_learned_read_modes_and_shapes(ds, dt):
    """The search's launch choices (each lane reading its own lines, or the blocks of X read by
    four lanes together; workgroup sizes) give the same exact indices, for the compiled router
    and the identity router."""
    rng = np.random.default_rng(29)
    X = _clustered(30_000, dt, 30_000)
    z = _queries(X, 70_001, rng)  # not a multiple of 64: the tail wave reads clamped queries
    ref = oracle.search(X, z)
    for epochs in (10, -1):
        idx = ds.build(_dev(X), method="learned", learn_epochs=epochs, learn_segments=1024, seed=4)
        for stage in (1, 2):
            for block in (256, 1024):
                idx.set_tune(stage=stage, block=block)
                _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref, z)
        _, fb = idx.learned_model()
        assert fb == 0
        idx.destroy()


def test_uniform_gaps_give_tight_windows(ds):
    """Closed form: X_i = i has a linear CDF, so every segment's fit is exact up to
    rounding and every window holds at most three candidates."""
    X = np.arange(0, 65537, dtype=np.float64)
    idx = ds.build(_dev(X), method="learned", learn_epochs=-1, learn_segments=1024)
    inf = idx.info()
    assert inf["max_err"] <= 1
    assert inf["mean_log2_window"] <= np.log2(3) + 1e-9
    z = np.concatenate([np.random.default_rng(1).uniform(0, 65536, 100_000), X, W.prev_float(X, np.float64)])
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z))


def test_auto_and_fallback_choose_learned_on_infeasible(ds):
    X = _clustered(20_000, np.float64, 3)
    X = np.unique(np.concatenate([X, [1.0, np.nextafter(1.0, 2.0)]]))  # one gap of 1 ulp: no feasible H
    assert oracle.compute_hr(X).status == oracle.ERR_INFEASIBLE
    z = _queries(X, 50_000, np.random.default_rng(2))
    ref = oracle.search(X, z)
    for kw in (dict(method="auto"), dict(fallback="learned")):
        idx = ds.build(_dev(X), learn_epochs=10, learn_segments=1024, **kw)
        assert idx.info()["method_name"] == "learned"
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), ref)
    # auto keeps Direct where it is feasible
    Xu = W.sweep_array(4096, np.float64)
    assert ds.build(_dev(Xu), method="auto").info()["method_name"] == "direct"


def test_network_gains_over_identity_router(ds):
    """What the trained router buys: narrower windows than equal-width segments of the feature."""
    X = W.clustered_array(1 << 17)
    trained = ds.build(_dev(X), method="learned", learn_segments=1024, learn_epochs=30).info()
    plain = ds.build(_dev(X), method="learned", learn_segments=1024, learn_epochs=-1).info()
    assert trained["mean_log2_window"] < plain["mean_log2_window"]


def test_full_size_clustered_f64_sampled(ds):
    """N + 1 = 2^20 lognormal draws, M = 2^26 (half uniform, half X_k (1 + 1e-12 noise))."""
    X = W.clustered_array()
    assert oracle.compute_hr(X).status == oracle.ERR_INFEASIBLE  # Direct table explodes
    z = W.clustered_queries(X, 1 << 26)
    X_d, z_d = _dev(X), _dev(z)
    idx = ds.build(X_d, method="learned")
    out = ds.search(idx, z_d)
    idx32 = ds.build(X_d, method="learned", learn_fp32_router=True)
    assert torch.equal(ds.search(idx32, z_d), out)
    torch.cuda.synchronize()
    i = out.long()
    assert int(i.min()) >= 0 and int(i.max()) <= X.size - 2
    assert bool(torch.all(X_d[i] <= z_d)) and bool(torch.all(z_d < X_d[i + 1]))
    pos = np.random.default_rng(3).integers(0, z.size, 1 << 18)
    _assert_same(out[torch.from_numpy(pos).to(DEV)].cpu().numpy(), oracle.search(X, z[pos]))
    _, fb = idx.learned_model()
    assert fb == 0
    torch.cuda.synchronize()
    inf = idx.info()
    assert inf["fallback_count"] == 0
    assert inf["model_bytes"] < 200_000
