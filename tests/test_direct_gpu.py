"""GPU parity of the single-array methods against the CPU oracle.

Every index is compared element by element with the oracle's classic binary
search; the Direct build's H, W, R, jmin and table K are compared bit for bit
with the oracle's ComputeHR/InitK.  At the full sweep size (2^26 queries, the
benchmark's launch configuration) outputs are sampled and the defining
invariant X_i <= z < X_{i+1} is checked for every query on the device.
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


def _check_tables(idx, X, form, hstart=oracle.HSTART_PHI):
    t = oracle.build_direct(X, FORMS[form], hstart)
    assert t.status == oracle.OK
    inf = idx.info()
    assert inf["method_name"] == "direct"
    assert inf["H"] == t.H and inf["W"] == t.W and inf["R"] == t.R and inf["jmin"] == t.jmin
    assert inf["n_h_updates"] == t.n_updates
    assert inf["fallback_count"] == 0 and inf["model_bytes"] == 0
    K = idx.table().cpu().numpy()
    assert np.array_equal(K, t.K)
    return t


def _queries(X, rng, m):
    """Uniform queries over [X_0, X_N), every key, the float below every key, and a few
    out-of-domain values."""
    dt = X.dtype
    zu = W.uniform_queries(X[0], X[-1], m, dt, rng)
    extra = np.array([np.nan, -np.inf, np.inf, X[-1], W.prev_float(X[:1], dt)[0]], dt)
    return np.concatenate([zu, X, W.prev_float(X, dt), extra]).astype(dt)


def _assert_same(got, ref, z=None):
    if not np.array_equal(got, ref):
        bad = np.flatnonzero(got != ref)
        extra = f" z={z[bad[:4]]}" if z is not None else ""
        raise AssertionError(f"{bad.size} of {ref.size} indices differ; first at {bad[:4]}: "
                             f"got {got[bad[:4]]} want {ref[bad[:4]]}{extra}")


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_plain_f32_1024_all_queries(ds, form):
    c = W.plain_f32_1024()
    z = np.concatenate([c.z_all, c.z_outside])
    idx = ds.build(_dev(c.X), form=form)
    _check_tables(idx, c.X, form)
    got = ds.search(idx, _dev(z)).cpu().numpy()
    _assert_same(got, oracle.search(c.X, z), z)
    # adversarial families explicitly
    n = c.N
    assert np.array_equal(ds.search(idx, _dev(c.z_hits)).cpu().numpy(), np.arange(n))
    assert np.array_equal(ds.search(idx, _dev(c.z_below)).cpu().numpy(), np.arange(n))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", W.SWEEP_N)
@pytest.mark.parametrize("form", ["sub", "fma"])
def test_sweep_tables_and_indices(ds, dtype, n, form):
    """Every layout the build can make, at every size of the sweep."""
    X = W.sweep_array(n, dtype)
    z = W.sweep_queries(1 << 20, dtype, stream=1)
    z = np.concatenate([z, X[:-1], W.prev_float(X[1:], dtype)[: 1 << 16], np.nextafter(X, np.dtype(dtype).type(2))])
    idx = ds.build(_dev(X), form=form, layouts=("rankcode", "pairs", "nibble"))
    _check_tables(idx, X, form)
    ref = oracle.search(X, z)
    z_d = _dev(z)
    for stage in _stages(idx):
        idx.set_tune(stage=stage)
        _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)
    idx.clear_tune()
    _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_mid_sizes_nibble_in_lds(ds, dtype):
    """Between RANKCODE's LDS limit (about 65,000 keys) and NIBBLE's (about 120,000) the automatic
    layout stages the NIBBLE chunks in LDS (stage 7); beyond, they are read through L2 (stage 6).
    Every layout, both forms and the fused histogram and interpolation agree with the oracle."""
    from oracle import apps

    rng = np.random.default_rng(12)
    for n, want in ((70_000, 7), (100_000, 7), (120_000, 7), (131_000, 6)):
        X = W.sweep_array(n, dtype)
        z = W.sweep_queries((1 << 19) + 5, dtype, stream=3)
        z = np.concatenate([z, X[:-1], W.prev_float(X[1:], dtype), np.nextafter(X, np.dtype(dtype).type(2))])
        ref = oracle.search(X, z)
        for form in ("sub", "fma"):
            idx = ds.build(_dev(X), form=form, layouts=("nibble",))
            inf = idx.info()
            assert inf["staged"] == want, (n, inf["staged"], inf["nibble_bytes"], inf["rankcode_bytes"])
            assert (inf["nibble_bytes"] <= 160 * 1024) == (want == 7)
            z_d = _dev(z)
            _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)
            for stage in _stages(idx):
                idx.set_tune(stage=stage)
                _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)
            idx.clear_tune()
            _assert_same(idx.histogram(z_d).cpu().numpy(), apps.histogram(X, z))
            Y = np.cumsum(rng.normal(0, 1, X.size)).astype(dtype)
            got = idx.interp_linear(_dev(Y), z_d).cpu().numpy()
            want_y = apps.interp_linear(X, Y, z)
            assert np.array_equal(got, want_y, equal_nan=True), (n, form)
            idx.destroy()


def _invariant_on_device(X_d, z_d, out_d):
    """X_i <= z < X_{i+1} for every query (all queries in [X_0, X_N))."""
    n = X_d.numel() - 1
    assert int(out_d.min()) >= 0 and int(out_d.max()) <= n - 1
    i = out_d.long()
    lo = X_d[i]
    hi = X_d[i + 1]
    assert bool(torch.all(lo <= z_d)) and bool(torch.all(z_d < hi))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", W.SWEEP_N)
def test_full_size_sweep_sampled(ds, dtype, n):
    """M = 2^26 in the benchmark's launch shape: sampled oracle check + invariant everywhere."""
    X = W.sweep_array(n, dtype)
    X_d = _dev(X)
    z_d = W.sweep_queries_torch(W.SWEEP_M, dtype, DEV)
    idx = ds.build(X_d)
    out = ds.search(idx, z_d)
    torch.cuda.synchronize()
    _invariant_on_device(X_d, z_d, out)
    g = torch.Generator(device="cpu").manual_seed(n)
    pos = torch.randint(0, W.SWEEP_M, (1 << 18,), generator=g).to(DEV)
    zs = z_d[pos].cpu().numpy()
    _assert_same(out[pos].cpu().numpy(), oracle.search(X, zs), zs)
    del out, z_d


@pytest.mark.parametrize("method", ["leadbit", "offset"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 255, 256, 257, 4096, 65536, 1 << 20])
def test_binary_search_baselines(ds, method, dtype, n):
    rng = np.random.default_rng(n)
    X = W.gap_array(n, dtype, rng, x0=-3.0)
    z = np.concatenate([W.uniform_queries(X[0], X[-1], 200_000, dtype, rng), X, W.prev_float(X, dtype),
                        np.nextafter(X, np.dtype(dtype).type(np.inf)),
                        np.array([np.nan, np.inf, -np.inf, 0.0, -0.0], dtype)]).astype(dtype)
    idx = ds.build(_dev(X), method=method)
    assert idx.info()["method_name"] == method
    got = ds.search(idx, _dev(z)).cpu().numpy()
    _assert_same(got, oracle.search(X, z), z)


def _stages(idx):
    inf = idx.info()
    if inf["method_name"] != "direct":
        return (1, 2) if inf["staged"] == 1 else (2,)
    st = [2]
    if inf["staged"] == 1:
        st.append(1)
    if inf["rankcode_bytes"] and inf["rankcode_bytes"] <= 160 * 1024 - 64:
        st.append(3)
    if inf["pairs_bytes"]:
        st.append(4)
    if inf["rankcode_bytes"]:
        st.append(5)
    if inf["nibble_bytes"]:
        st.append(6)
    if inf["nibble_bytes"] and inf["nibble_bytes"] <= 160 * 1024:
        st.append(7)
    return tuple(sorted(st))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_every_launch_shape_gives_the_same_answer(ds, dtype):
    for n in (256, 65536):
        X = W.sweep_array(n, dtype)
        z = W.sweep_queries((1 << 18) + 3, dtype, stream=2)
        ref = oracle.search(X, z)
        for method in ("direct", "leadbit"):
            idx = ds.build(_dev(X), method=method, layouts=("rankcode", "pairs", "nibble") if method == "direct" else ())
            z_d = _dev(z)
            stages = _stages(idx)
            if method == "direct":
                assert 4 in stages and 5 in stages and (3 in stages) == (n <= 65536)
            for stage in stages:
                for block in (64, 256, 1024):
                    for unroll in (1, 2, 4):
                        for grid in (0, 1, 7):
                            idx.set_tune(block=block, unroll=unroll, stage=stage, grid=grid)
                            got = ds.search(idx, z_d).cpu().numpy()
                            _assert_same(got, ref)
            idx.clear_tune()


def test_autotune_keeps_results(ds):
    for dt in (np.float32, np.float64):
        for n in (16, 65536, 1 << 20):
            X = W.sweep_array(n, dt)
            z_d = W.sweep_queries_torch(1 << 21, dt, DEV, stream=5)
            idx = ds.build(_dev(X), layouts=("rankcode", "pairs", "nibble"))
            ref = ds.search(idx, z_d).clone()
            best = idx.autotune(z_d)
            assert best["stage"] in _stages(idx)
            assert torch.equal(ds.search(idx, z_d), ref)
            zs = z_d[:100_000].cpu().numpy()
            _assert_same(ref[:100_000].cpu().numpy(), oracle.search(X, zs))


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_ragged_and_unaligned_sizes(ds, form):
    X = W.sweep_array(4096, np.float64)
    idx = ds.build(_dev(X), form=form)
    zall = W.sweep_queries(5000, np.float64, stream=3)
    ref = oracle.search(X, zall)
    z_d = _dev(zall)
    for m in (0, 1, 2, 3, 4, 5, 7, 63, 64, 65, 1023, 4097):
        for off in (0, 1, 3):
            if off + m > zall.size:
                continue
            zz = z_d[off:off + m]
            out = torch.empty(m + 1, dtype=torch.int32, device=DEV)[1:]  # misaligned output
            got = ds.search(idx, zz.contiguous() if off == 0 else zz, out=out).cpu().numpy()
            _assert_same(got, ref[off:off + m])


def test_exhaustive_f32_domain_on_gpu(ds):
    """Every f32 value in [X_0, X_N) for X inside 2^22 consecutive floats above 1.0."""
    span = (np.array([1.0], np.float32).view(np.int32)[0] + np.arange(1 << 22, dtype=np.int32)).view(np.float32)
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(span.size - 2, size=500, replace=False)) + 1
    X = np.concatenate([[span[0]], span[pick], [span[-1]]]).astype(np.float32)
    z = span[:-1]
    ref = oracle.search(X, z)
    z_d = _dev(z)
    for form in ("sub", "fma"):
        idx = ds.build(_dev(X), form=form, layouts=("rankcode", "pairs", "nibble"))
        _check_tables(idx, X, form)
        for stage in _stages(idx):
            idx.set_tune(stage=stage)
            _assert_same(ds.search(idx, z_d).cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dense_neighbourhoods_all_layouts(ds, dtype):
    """All floats within 2^12 ulps of every X_i of a sweep array, through every layout."""
    dt = np.dtype(dtype)
    X = W.sweep_array(4096, dt)
    it = np.int32 if dt == np.float32 else np.int64
    offs = np.arange(-(1 << 12), 1 << 12, dtype=it)
    z = (X.view(it)[:, None] + offs[None, :]).reshape(-1).view(dt)
    z = z[np.isfinite(z)]
    ref = oracle.search(X, z)
    z_d = _dev(z)
    for form in ("sub", "fma"):
        idx = ds.build(_dev(X), form=form, layouts=("rankcode", "pairs", "nibble"))
        for stage in _stages(idx):
            idx.set_tune(stage=stage)
            _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)


def test_fma_form_with_negative_first_cell(ds):
    """Arrays at random offsets, where W = m(H X_0) can leave f(X_0) = -1."""
    rng = np.random.default_rng(9)
    seen = set()
    for k in range(60):
        X = W.gap_array(int(rng.integers(8, 3000)), np.float32, rng, x0=rng.uniform(-1e3, 1e3))
        t = oracle.build_direct(X, oracle.FORM_FMA)
        seen.add(t.jmin)
        idx = ds.build(_dev(X), form="fma", layouts=("rankcode", "pairs", "nibble"))
        _check_tables(idx, X, "fma")
        z = np.concatenate([W.uniform_queries(X[0], X[-1], 5000, np.float32, rng), X,
                            W.prev_float(X, np.float32), np.nextafter(X, np.float32(np.inf)),
                            np.array([np.nan, -np.inf, np.inf], np.float32)])
        ref = oracle.search(X, z)
        z_d = _dev(z)
        for stage in _stages(idx):
            idx.set_tune(stage=stage)
            _assert_same(ds.search(idx, z_d).cpu().numpy(), ref, z)
    assert -1 in seen and 0 in seen


def test_h_growth_matches_oracle(ds):
    """Start at Hbar so that ComputeHR must grow H now and then; H, updates and K match."""
    rng = np.random.default_rng(2024)
    grown = 0
    for a in range(6000):
        X = np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 5.0, 15))]).astype(np.float32)
        t = oracle.compute_hr(X, hstart=oracle.HSTART_HBAR)
        if t.n_updates == 0 and a % 200:
            continue
        grown += t.n_updates > 0
        for form in ("sub", "fma"):
            idx = ds.build(_dev(X), form=form, hstart="hbar")
            _check_tables(idx, X, form, oracle.HSTART_HBAR)
    assert grown > 0


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_small_build_growth_and_large_tables(ds, form):
    """The one-launch build of arrays up to 65537 values: near-limit arrays where ComputeHR
    grows H 16 to 23 times, offset or not, and arrays whose table exceeds the room kept
    beside X (max(4 (N + 1), 16384) cells) and gets its own allocation: H, W, R, jmin, the
    update count and K equal the oracle's, and so does every search."""
    rng = np.random.default_rng(91)
    grown = 0
    for a in range(60):
        X = W.near_limit_array(np.float32, rng, q=int(rng.integers(1, 4)), n_fill=int(rng.integers(0, 3000)),
                               offset=bool(a % 2))
        t = oracle.build_direct(X, FORMS[form])
        if t.status != oracle.OK:
            with pytest.raises(ds.DsError) as e:
                ds.build(_dev(X), form=form)
            assert e.value.status == t.status
            continue
        grown += t.n_updates > 0
        idx = ds.build(_dev(X), form=form)
        _check_tables(idx, X, form)
        z = _queries(X, rng, 20_000)
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z), z)
        idx.destroy()
    assert grown >= 10
    for n, spread in ((100, 1e-3), (3000, 1e-4), (65536, 1e-2)):
        # one tiny gap among unit gaps: R is about N / spread, far beyond 4 (N + 1) cells
        X = np.arange(n + 1, dtype=np.float64)
        X[1] = spread
        t = oracle.build_direct(X, FORMS[form])
        assert t.status == oracle.OK and t.R - t.jmin + 1 > max(4 * (n + 1), 16384)
        idx = ds.build(_dev(X), form=form)
        _check_tables(idx, X, form)
        z = _queries(X, rng, 20_000)
        _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z), z)
        idx.destroy()


def test_errors_and_fallback(ds):
    for case in ([-1e9, 0.0, 1.0], [0.0, 1.42e-45, 1.0]):  # Sec. 4.4
        with pytest.raises(ds.DsError) as e:
            ds.build(_dev(np.array(case, np.float32)))
        assert e.value.status == ds.ERR_INFEASIBLE
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(np.array([0, 1, 1, 2], np.float32)))
    assert e.value.status == ds.ERR_NOT_SORTED
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(np.array([0, 1, np.nan, 2], np.float64)))
    assert e.value.status == ds.ERR_NONFINITE
    X = W.sweep_array(65536, np.float32)
    with pytest.raises(ds.DsError) as e:
        ds.build(_dev(X), table_cap_bytes=1024)
    assert e.value.status == ds.ERR_TABLE_CAP
    idx = ds.build(_dev(X), table_cap_bytes=1024, fallback="bsearch")
    assert idx.info()["method_name"] == "leadbit"
    z = W.sweep_queries(100_000, np.float32)
    _assert_same(ds.search(idx, _dev(z)).cpu().numpy(), oracle.search(X, z))
    idx = ds.build(_dev(np.array([-1e9, 0.0, 1.0], np.float32)), fallback="bsearch")
    zz = np.array([-2e9, -1e9, -1.0, 0.0, 0.5, 1.0, 2.0], np.float32)
    _assert_same(ds.search(idx, _dev(zz)).cpu().numpy(), oracle.search(np.array([-1e9, 0.0, 1.0], np.float32), zz))


def test_graph_replay_matches_eager(ds):
    X = W.sweep_array(4096, np.float32)
    idx = ds.build(_dev(X))
    z_d = W.sweep_queries_torch(1 << 22, np.float32, DEV)
    eager = ds.search(idx, z_d).clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ds.search(idx, z_d, out=out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ds.search(idx, z_d, out=out)
    for r in range(4):
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        ds.search(idx, z_d[: 1000])  # eager work between replays


def test_maximum_sizes_int64_query_offsets_and_large_n(ds):
    """M = 2^31 + 4099 queries (offsets past int32 in the streaming loops, a ragged tail) on
    an LDS-resident table, and N = 2^25 f64 (its NIBBLE table, 22 MB, spills past L2):
    sampled against the oracle, including the last queries, plus the invariant on chunks."""
    X = W.sweep_array(4096, np.float32)
    xd = _dev(X)
    M = (1 << 31) + 4099
    g = torch.Generator(device=DEV)
    g.manual_seed(77)
    z = torch.rand(M, generator=g, device=DEV, dtype=torch.float32)
    idx = ds.build(xd)
    out = ds.search(idx, z)
    pos = np.concatenate([np.random.default_rng(1).integers(0, M, 1 << 16), np.arange(M - 4200, M)])
    pt = torch.from_numpy(pos).to(DEV)
    zs = z[pt].cpu().numpy()
    _assert_same(out[pt].cpu().numpy(), oracle.search(X, zs), zs)
    for c0 in range(0, M, 1 << 28):  # invariant on every query, chunk by chunk
        o = out[c0:c0 + (1 << 28)].long()
        zz = z[c0:c0 + (1 << 28)]
        assert int(o.min()) >= 0 and int(o.max()) <= X.size - 2
        assert bool(torch.all(xd[o] <= zz)) and bool(torch.all(zz < xd[o + 1]))
    del z, out, o, zz
    torch.cuda.empty_cache()
    n = 1 << 25
    Xb = W.sweep_array(n, np.float64)
    xb = _dev(Xb)
    idx = ds.build(xb)
    inf = idx.info()
    assert inf["staged"] == 6 and inf["nibble_bytes"] > (16 << 20)
    zb = W.sweep_queries_torch(1 << 26, np.float64, DEV)
    ob = ds.search(idx, zb)
    o = ob.long()
    assert bool(torch.all(xb[o] <= zb)) and bool(torch.all(zb < xb[o + 1]))
    pos = torch.from_numpy(np.random.default_rng(2).integers(0, 1 << 26, 1 << 16)).to(DEV)
    zs = zb[pos].cpu().numpy()
    _assert_same(ob[pos].cpu().numpy(), oracle.search(Xb, zs), zs)
