"""GPU parity of the batched ragged search against the CPU oracle.

Each array's outputs are compared element by element with the oracle's classic
binary search on that array; at the full size of the 10,000-array workload the
outputs are sampled and the defining invariant is checked for every query on
the device.
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


def _oracle_batch(x_off, X, q_off, z):
    ref = np.empty(z.size, np.int32)
    for k in range(x_off.size - 1):
        xa = X[x_off[k]:x_off[k + 1]]
        q0, q1 = q_off[k], q_off[k + 1]
        if q1 == q0:
            continue
        if xa.size == 0:
            ref[q0:q1] = -1
        else:
            ref[q0:q1] = oracle.search(xa, z[q0:q1])
    return ref


def _run(ds, b: W.Batch, **kw):
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z), **kw)
    out = bt.run().cpu().numpy()
    return bt, out


def _assert_same(got, ref):
    if not np.array_equal(got, ref):
        bad = np.flatnonzero(got != ref)
        raise AssertionError(f"{bad.size} of {ref.size} differ; first at {bad[:5]}: got {got[bad[:5]]} "
                             f"want {ref[bad[:5]]}")


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_small_batch_f32(ds, form):
    b = W.batched_f32(num_arrays=300, n_lo=8, n_hi=8192, q_per_n=16, seed=7)
    bt, out = _run(ds, b, form=form)
    _assert_same(out, _oracle_batch(b.x_off, b.X, b.q_off, b.z))
    meth, R = bt.report()
    assert np.all(meth == ds.METHOD_DIRECT)
    # per-array R equals the oracle's ComputeHR
    for k in range(0, 300, 37):
        t = oracle.compute_hr(b.array(k), oracle.FORM_SUB if form == "sub" else oracle.FORM_FMA)
        assert t.R == R[k]


def test_batch_equals_single_array_search(ds):
    b = W.batched_f32(num_arrays=40, n_lo=8, n_hi=65536, q_per_n=8, seed=8)
    _, out = _run(ds, b)
    for k in range(b.num_arrays):
        idx = ds.build(_dev(b.array(k)))
        single = ds.search(idx, _dev(b.queries(k))).cpu().numpy()
        assert np.array_equal(out[b.q_off[k]:b.q_off[k + 1]], single), k


def test_batch_f64_mixture_small(ds):
    rng = np.random.default_rng(4)
    arrays = [W.mixture_array(int(n), rng) for n in (100, 2000, 30000, 70000)]
    X = np.concatenate(arrays)
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    zs = [W.mixture_queries(a, 50_000, rng) for a in arrays]
    z = np.concatenate(zs)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    bt, out = _run(ds, W.Batch(np.dtype(np.float64), x_off, X, q_off, z))
    _assert_same(out, _oracle_batch(x_off, X, q_off, z))
    meth, _ = bt.report()
    # clustered arrays are infeasible for Direct and fall back to binary search
    assert set(meth.tolist()) <= {ds.METHOD_DIRECT, ds.METHOD_BSEARCH_OFFSET}


def test_edge_arrays(ds):
    f32 = np.float32
    arrays = [
        np.array([], f32),                       # N = -1: no value
        np.array([5.0], f32),                    # N = 0: one value
        np.array([0.0, 1.0], f32),               # N = 1
        np.array([-1e9, 0.0, 1.0], f32),         # infeasible (Sec. 4.4): binary search
        np.array([0.0, 1.42e-45, 1.0], f32),     # infeasible (overflow of 1/min gap)
        np.array([0.0, 2.0, 1.0], f32),          # not sorted: -2
        np.array([0.0, np.nan, 1.0], f32),       # not finite: -2
        W.gap_array(1000, f32, np.random.default_rng(1), x0=-7.0),
        W.gap_array(5, f32, np.random.default_rng(2)),   # no queries
    ]
    rng = np.random.default_rng(3)
    zs = []
    for k, a in enumerate(arrays):
        if k == 8:
            zs.append(np.array([], f32))
            continue
        lo, hi = (float(a[0]) - 2, float(a[-1]) + 2) if a.size else (-1, 1)
        zz = rng.uniform(lo, hi, 3000).astype(f32)
        extra = np.concatenate([a, W.prev_float(a, f32), np.array([np.nan, np.inf, -np.inf], f32)]) if a.size else \
            np.array([0.0, np.nan], f32)
        zs.append(np.concatenate([zz, extra[np.isfinite(extra) | np.isnan(extra) | np.isinf(extra)]]).astype(f32))
    X = np.concatenate(arrays).astype(f32)
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    z = np.concatenate(zs).astype(f32)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    bt, out = _run(ds, W.Batch(np.dtype(f32), x_off, X, q_off, z))
    meth, _ = bt.report()
    assert meth.tolist() == [-2, -2, 0, 2, 2, -1, -1, 0, 0]
    for k in range(len(arrays)):
        got = out[q_off[k]:q_off[k + 1]]
        if k in (5, 6):
            assert np.all(got == -2)
            continue
        ref = _oracle_batch(x_off[k:k + 2] - x_off[k], arrays[k], q_off[k:k + 2] - q_off[k], zs[k])
        _assert_same(got, ref)


def _growth_batch(rng, dt):
    """Arrays where ComputeHR grows H two or more times (at the feasibility limit, with and
    without filler keys), mixed with empty, one-value, tiny, mid-sized, infeasible and
    unsorted arrays in random order, so that the build's 4096-value scan chunks start and end
    inside arrays, at their ends and among runs of tiny arrays."""
    arrays = []
    # four chosen by growth in the subtraction form, four in the FMA form, four in the FMA
    # form with X_0 < 0 (growth there is rarer: bounded tries)
    for form, offset in ((oracle.FORM_SUB, False), (oracle.FORM_FMA, False), (oracle.FORM_FMA, True)):
        found = 0
        for _ in range(40_000):
            X = W.near_limit_array(dt, rng, n_fill=int(rng.integers(0, 6000)), offset=offset)
            t = oracle.compute_hr(X, form)
            if t.status == oracle.OK and t.n_updates >= 2 and t.R < (1 << 26):
                arrays.append(X)
                found += 1
                if found == 4:
                    break
        assert found == 4
    for _ in range(10):
        arrays.append(np.array([], dt))
        arrays.append(np.array([rng.uniform(-5, 5)], dt))
        arrays.append(W.gap_array(int(rng.integers(1, 40)), dt, rng, x0=rng.uniform(-100, 100)))
    for _ in range(6):
        arrays.append(W.gap_array(int(rng.integers(3000, 20000)), dt, rng, x0=rng.uniform(-100, 100)))
    arrays.append(np.array([-1e9, 0.0, 1.0], dt))   # infeasible
    arrays.append(np.array([0.0, 2.0, 1.0], dt))    # not increasing
    order = rng.permutation(len(arrays))
    arrays = [arrays[i] for i in order]
    zs = []
    for a in arrays:
        if a.size == 0:
            zs.append(np.array([0.0, np.nan], dt))
            continue
        u = rng.uniform(float(a[0]) - 1, float(a[-1]) + 1, 2000).astype(dt)
        zs.append(np.concatenate([u, a, W.prev_float(a, dt), np.array([np.nan, np.inf, -np.inf], dt)]).astype(dt))
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    return arrays, W.Batch(np.dtype(dt), x_off, np.concatenate(arrays).astype(dt), q_off, np.concatenate(zs))


@pytest.mark.parametrize("form", ["sub", "fma"])
def test_batched_build_growth_and_chunk_edges(ds, form):
    """Per array the device build's method and R equal the oracle's ComputeHR (H grown up to
    the float of the sequential algorithm), and every result equals the oracle's search; the
    same from an X pointer that is not 16-byte aligned (the build reads it with scalar loads)."""
    rng = np.random.default_rng(21)
    arrays, b = _growth_batch(rng, np.float32)
    budget = 1 << 29
    bt, out = _run(ds, b, form=form, table_budget_entries=budget)
    meth, R = bt.report()
    fm = oracle.FORM_SUB if form == "sub" else oracle.FORM_FMA
    grown = 0
    for k, a in enumerate(arrays):
        if a.size <= 1:
            assert meth[k] == -2, k
            continue
        if not np.all(a[1:] > a[:-1]):
            assert meth[k] == -1, k
            continue
        t = oracle.compute_hr(a, fm)
        if t.status == oracle.OK and t.R < (1 << 26):
            assert meth[k] == ds.METHOD_DIRECT and R[k] == t.R, (k, a.size, meth[k], R[k], t.R)
            grown += t.n_updates >= 2
        elif t.status != oracle.OK:
            assert meth[k] == ds.METHOD_BSEARCH_OFFSET, k
    assert grown >= 8
    ref = _oracle_batch(b.x_off, b.X, b.q_off, b.z)
    bad = [k for k, a in enumerate(arrays) if a.size > 1 and not np.all(a[1:] > a[:-1])]
    for k in bad:
        assert np.all(out[b.q_off[k]:b.q_off[k + 1]] == -2)
        ref[b.q_off[k]:b.q_off[k + 1]] = -2
    _assert_same(out, ref)
    # the same batch from a pointer 4 bytes past a 16-byte boundary
    pad = torch.empty(b.X.size + 1, dtype=torch.float32, device=DEV)
    pad[1:] = _dev(b.X)
    Xu = pad[1:]
    assert Xu.data_ptr() % 16 == 4
    bt2 = ds.Batch(_dev(b.x_off), Xu, _dev(b.q_off), _dev(b.z), form=form, table_budget_entries=budget)
    _assert_same(bt2.run().cpu().numpy(), out)
    meth2, R2 = bt2.report()
    assert np.array_equal(meth2, meth) and np.array_equal(R2, R)


def test_many_tiny_arrays_per_chunk(ds):
    """20,000 arrays of 0 to 12 values: the build's 4096-value chunks hold about 2,000 arrays
    each in the first half (more than its 1,024 LDS slots: per-lane global atomics) and about
    500 in the second (merged in LDS); every result equals the oracle's search."""
    rng = np.random.default_rng(31)
    f32 = np.float32
    sizes = np.concatenate([rng.integers(0, 5, 10_000), rng.integers(3, 13, 10_000)])
    arrays, zs = [], []
    for n in sizes:
        a = W.gap_array(int(n) - 1, f32, rng, x0=rng.uniform(-50, 50)) if n > 0 else np.array([], f32)
        arrays.append(a)
        lo, hi = (float(a[0]) - 1, float(a[-1]) + 1) if a.size else (-1.0, 1.0)
        zs.append(np.concatenate([rng.uniform(lo, hi, 6).astype(f32), a]).astype(f32))
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    b = W.Batch(np.dtype(f32), x_off, np.concatenate(arrays).astype(f32), q_off, np.concatenate(zs))
    for form in ("sub", "fma"):
        bt, out = _run(ds, b, form=form)
        meth, _ = bt.report()
        assert np.all(meth[sizes <= 1] == -2) and np.all(meth[sizes >= 2] == ds.METHOD_DIRECT)
        _assert_same(out, _oracle_batch(x_off, b.X, q_off, b.z))


@pytest.mark.parametrize("learn", [0, 64])
def test_batches_without_keys_or_queries(ds, learn):
    """Every array empty (no packed key at all: the build's chunked passes have nothing to
    scan), and a batch with keys but no query; with and without learned models."""
    f32 = np.float32
    x_off = np.zeros(4, np.int64)
    q_off = np.array([0, 3, 3, 5], np.int64)
    z = np.array([0.0, np.nan, -1.0, 2.0, np.inf], f32)
    bt = ds.Batch(_dev(x_off), torch.empty(0, dtype=torch.float32, device=DEV), _dev(q_off), _dev(z),
                  learn_segments=learn)
    assert np.all(bt.run().cpu().numpy() == -1)
    meth, _ = bt.report()
    assert np.all(meth == -2)
    b = W.batched_f32(num_arrays=20, n_lo=8, n_hi=3000, q_per_n=1, seed=15)
    q_none = np.zeros(21, np.int64)
    bt2 = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(q_none), torch.empty(0, dtype=torch.float32, device=DEV),
                   learn_segments=learn)
    assert bt2.run().numel() == 0
    meth2, R2 = bt2.report()
    assert np.all(meth2 == ds.METHOD_DIRECT)
    for k in range(0, 20, 7):
        assert R2[k] == oracle.compute_hr(b.array(k)).R


def test_no_table_room_uses_binary_search(ds):
    b = W.batched_f32(num_arrays=50, n_lo=8, n_hi=20000, q_per_n=8, seed=9)
    bt, out = _run(ds, b, table_budget_entries=0)
    meth, _ = bt.report()
    assert np.all(meth == ds.METHOD_BSEARCH_OFFSET)
    _assert_same(out, _oracle_batch(b.x_off, b.X, b.q_off, b.z))
    # partial room: a prefix of the arrays gets Direct
    bt2, out2 = _run(ds, b, table_budget_entries=int(np.sum(np.diff(b.x_off))) // 2)
    meth2, _ = bt2.report()
    assert (meth2 == ds.METHOD_DIRECT).any() and (meth2 == ds.METHOD_BSEARCH_OFFSET).any()
    _assert_same(out2, out)


def test_every_launch_shape_gives_the_same_answer(ds):
    b = W.batched_f32(num_arrays=120, n_lo=8, n_hi=65536, q_per_n=4, seed=10)
    ref = _oracle_batch(b.x_off, b.X, b.q_off, b.z)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z))
    for tile in (1000, 1 << 16, 1 << 19):
        for block in (256, 1024):
            for qpt in (4, 8, 16):
                for lds in (0, -1, 40_000):
                    bt.set_shape(tile=tile, block=block, lds_bytes=lds, qpt=qpt)
                    out = bt.run().cpu().numpy()
                    _assert_same(out, ref)


def test_autotune_keeps_results(ds, tmp_path):
    b = W.batched_f32(num_arrays=150, n_lo=8, n_hi=65536, q_per_n=16, seed=13)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z))
    ref = bt.run().cpu().numpy()
    cache = str(tmp_path / "tune.json")
    best = bt.autotune(cache=cache)
    assert best["tile"] in (1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20) and best["qpt"] in (4, 8, 16)
    assert np.array_equal(bt.run().cpu().numpy(), ref)
    bt2 = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z))
    assert bt2.autotune(cache=cache) == best  # served from the cache
    _assert_same(ref, _oracle_batch(b.x_off, b.X, b.q_off, b.z))


def test_autotune_with_tables_out_of_room(ds):
    """The autotuner re-plans the query tiles for each candidate shape; arrays that the first
    plan moved to binary search for lack of table room keep their method and the others keep
    their table offsets, so the output it leaves equals the oracle's."""
    b = W.batched_f32(num_arrays=80, n_lo=8, n_hi=20000, q_per_n=8, seed=14)
    ref = _oracle_batch(b.x_off, b.X, b.q_off, b.z)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z),
                  table_budget_entries=int(np.sum(np.diff(b.x_off))) // 2)
    _assert_same(bt.run().cpu().numpy(), ref)
    meth, _ = bt.report()
    assert (meth == ds.METHOD_DIRECT).any() and (meth == ds.METHOD_BSEARCH_OFFSET).any()
    bt.autotune()
    _assert_same(bt.out.cpu().numpy(), ref)   # the last candidate's search
    meth2, _ = bt.report()
    assert np.array_equal(meth2, meth)
    _assert_same(bt.run().cpu().numpy(), ref)


def test_graph_capture_replays(ds):
    b = W.batched_f32(num_arrays=200, n_lo=8, n_hi=65536, q_per_n=8, seed=11)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z))
    eager = bt.run().clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    for r in range(4):
        bt.out.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bt.out, eager), r
        bt.run()  # eager work between replays
        torch.cuda.synchronize()
    _assert_same(eager.cpu().numpy(), _oracle_batch(b.x_off, b.X, b.q_off, b.z))


def test_graph_capture_replays_learned(ds):
    """A batch whose arrays take the learned method (device build, training steps, routing, fits
    and search, all captured): every replay equals the eager run and the oracle."""
    b = _mixture_batch((3000, 9000, 20000, 500), 20_000, 12)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z), learn_segments=512, learn_steps=8,
                  direct_cap_bytes=64)
    eager = bt.run().clone()
    meth, _ = bt.report()
    assert np.all(meth == ds.METHOD_LEARNED)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    for r in range(4):
        bt.out.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bt.out, eager), r
        bt.run()  # eager work between replays
        torch.cuda.synchronize()
    _assert_same(eager.cpu().numpy(), _oracle_batch(b.x_off, b.X, b.q_off, b.z))
    assert bt.fallbacks() == 0


def test_full_size_batched_f32_sampled(ds):
    """10,000 arrays, N_k log-uniform in [8, 65536], M_k = 64 N_k (about 4.5e9 queries)."""
    b = W.batched_f32(with_queries=False)
    total_q = int(b.q_off[-1])
    assert total_q > 2**32  # int64 offsets are exercised
    z = W.batched_queries_torch(b, DEV)
    x_off_d, X_d, q_off_d = _dev(b.x_off), _dev(b.X), _dev(b.q_off)
    bt = ds.Batch(x_off_d, X_d, q_off_d, z)
    out = bt.run()
    torch.cuda.synchronize()
    meth, _ = bt.report()
    assert np.all(meth == ds.METHOD_DIRECT)
    # invariant X_i <= z < X_{i+1} for every query, array chunk by array chunk
    for a in range(0, b.num_arrays, 500):
        e = min(b.num_arrays, a + 500)
        q0, q1 = int(b.q_off[a]), int(b.q_off[e])
        counts = torch.from_numpy(np.diff(b.q_off[a:e + 1])).to(DEV)
        base = torch.repeat_interleave(x_off_d[a:e], counts)
        nk = torch.repeat_interleave(x_off_d[a + 1:e + 1] - x_off_d[a:e] - 1, counts)
        i = out[q0:q1].long()
        assert bool(torch.all((i >= 0) & (i < nk)))
        zz = z[q0:q1]
        assert bool(torch.all(X_d[base + i] <= zz)) and bool(torch.all(zz < X_d[base + i + 1]))
        del counts, base, nk, i
    # sampled oracle check
    g = torch.Generator(device="cpu").manual_seed(12)
    pos = torch.randint(0, total_q, (1 << 18,), generator=g).numpy()
    pos.sort()
    zs = z[torch.from_numpy(pos).to(DEV)].cpu().numpy()
    got = out[torch.from_numpy(pos).to(DEV)].cpu().numpy()
    ks = np.searchsorted(b.q_off, pos, side="right") - 1
    ref = np.empty_like(got)
    for k in np.unique(ks):
        sel = ks == k
        ref[sel] = oracle.search(b.array(k), zs[sel])
    _assert_same(got, ref)


def _mixture_batch(ns, m_each, seed):
    rng = np.random.default_rng(seed)
    arrays = [W.mixture_array(int(n), rng) for n in ns]
    X = np.concatenate(arrays)
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    zs = [W.mixture_queries(a, m_each, rng) for a in arrays]
    z = np.concatenate(zs)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    return W.Batch(np.dtype(np.float64), x_off, X, q_off, z)


def test_batched_learned_no_network_exact(ds):
    """The ablation of the batched router (learn_steps = -1: segments split the feature evenly,
    no training) keeps the results of the trained models, exactly."""
    b = _mixture_batch((500, 3000, 20000, 7), 30_000, 24)
    ref = _oracle_batch(b.x_off, b.X, b.q_off, b.z)
    for steps in (-1, 3):
        bt, out = _run(ds, b, learn_segments=1024, learn_steps=steps, direct_cap_bytes=64)
        meth, _ = bt.report()
        assert np.all(meth[np.diff(b.x_off) > 1] == ds.METHOD_LEARNED)
        _assert_same(out, ref)
        assert bt.fallbacks() == 0


def test_batched_learned_mixture_exact(ds):
    b = _mixture_batch((300, 2000, 9000, 40000, 70000, 5), 60_000, 21)
    bt, out = _run(ds, b, learn_segments=1024, learn_steps=60)
    meth, _ = bt.report()
    assert (meth == ds.METHOD_LEARNED).any()
    assert set(meth.tolist()) <= {ds.METHOD_DIRECT, ds.METHOD_LEARNED}
    _assert_same(out, _oracle_batch(b.x_off, b.X, b.q_off, b.z))
    assert bt.fallbacks() == 0
    # forcing every array off Direct with a tiny per-array cap keeps the results
    bt2, out2 = _run(ds, b, learn_segments=512, learn_steps=20, direct_cap_bytes=64)
    meth2, _ = bt2.report()
    assert np.all((meth2 == ds.METHOD_LEARNED))
    _assert_same(out2, out)
    assert bt2.fallbacks() == 0


def test_batched_learned_f32_and_shapes(ds):
    b = W.batched_f32(num_arrays=30, n_lo=8, n_hi=30000, q_per_n=8, seed=22)
    ref = _oracle_batch(b.x_off, b.X, b.q_off, b.z)
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z), learn_segments=256, learn_steps=10,
                  direct_cap_bytes=4 * 4096)
    for tile in (1000, 1 << 16):
        bt.set_shape(tile=tile)
        _assert_same(bt.run().cpu().numpy(), ref)
    meth, _ = bt.report()
    assert (meth == ds.METHOD_LEARNED).any() and (meth == ds.METHOD_DIRECT).any()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_learned_block_scan_at_buffer_edges(ds, dtype):
    """The learned search reads 64-byte blocks aligned in memory: arrays at unaligned offsets,
    a packed buffer that itself starts off a 64-byte boundary (a view one value into a larger
    tensor), and queries packed at both ends of every array, the last array's end being the
    end of the buffer."""
    rng = np.random.default_rng(31)
    sizes = [5, 17, 300, 2500, 40, 9000, 3]
    arrays = [W.gap_array(n, dtype, rng, x0=rng.uniform(-50, 50)) for n in sizes]
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    X = np.concatenate(arrays).astype(dtype)
    zs = []
    for a in arrays:
        ends = np.concatenate([a[:12], a[-12:]])
        zs.append(np.concatenate([ends, W.prev_float(ends, dtype), np.nextafter(ends, dtype(np.inf)),
                                  W.uniform_queries(a[0], a[-1], 500, dtype, rng),
                                  np.array([a[0] - 1, a[-1] + 1, np.nan], dtype)]).astype(dtype))
    z = np.concatenate(zs)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    ref = _oracle_batch(x_off, X, q_off, z)
    big = torch.zeros(X.size + 1, dtype=torch.float32 if dtype == np.float32 else torch.float64, device=DEV)
    big[1:] = _dev(X)
    Xv = big[1:]  # starts 4 or 8 bytes past an allocation boundary
    for segs in (64, 1024):
        bt = ds.Batch(_dev(x_off), Xv, _dev(q_off), _dev(z), learn_segments=segs, learn_steps=10,
                      direct_cap_bytes=8)
        out = bt.run().cpu().numpy()
        meth, _ = bt.report()
        assert np.all(meth == ds.METHOD_LEARNED)
        _assert_same(out, ref)
        assert bt.fallbacks() == 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_learned_segment_counts_off_four(ds, dtype):
    """Segment counts that are not multiples of 4 (1, 3, 5, 37, 1023): each model's step table
    and grid then start off a 16-byte boundary in the workspace and in LDS, and the fit kernel's
    last group of segments is partial.  Exact results without fallback, trained and without
    network."""
    rng = np.random.default_rng(37)
    sizes = [9, 700, 5000, 20_000, 64]
    arrays = [W.gap_array(n, dtype, rng, x0=rng.uniform(-50, 50)) for n in sizes]
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    X = np.concatenate(arrays).astype(dtype)
    zs = [np.concatenate([a[:8], W.prev_float(a[-8:], dtype), W.uniform_queries(a[0], a[-1], 3000, dtype, rng)])
          .astype(dtype) for a in arrays]
    z = np.concatenate(zs)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    ref = _oracle_batch(x_off, X, q_off, z)
    for segs in (1, 3, 5, 37, 1023):
        for steps in (6, -1):
            bt = ds.Batch(_dev(x_off), _dev(X), _dev(q_off), _dev(z), learn_segments=segs, learn_steps=steps,
                          direct_cap_bytes=8)
            out = bt.run().cpu().numpy()
            meth, _ = bt.report()
            assert np.all(meth == ds.METHOD_LEARNED)
            _assert_same(out, ref)
            assert bt.fallbacks() == 0


def test_full_size_batched_learned_f64_sampled(ds):
    """256 mixture arrays, N_k log-uniform in [2^14, 2^20], 2^28 queries (70 % uniform, 20 % hits,
    10 % nextafter(X_i, -inf)); Direct where its table fits under 64 MB, the learned method elsewhere."""
    b = W.batched_mixture(with_queries=False)
    z = W.batched_mixture_queries_torch(b, DEV)
    x_off_d, X_d, q_off_d = _dev(b.x_off), _dev(b.X), _dev(b.q_off)
    bt = ds.Batch(x_off_d, X_d, q_off_d, z, learn_segments=4096, direct_cap_bytes=64 << 20)
    out = bt.run()
    torch.cuda.synchronize()
    meth, _ = bt.report()
    assert set(meth.tolist()) <= {ds.METHOD_DIRECT, ds.METHOD_LEARNED}
    assert bt.fallbacks() == 0
    for a in range(0, b.num_arrays, 32):
        e = min(b.num_arrays, a + 32)
        q0, q1 = int(b.q_off[a]), int(b.q_off[e])
        counts = torch.from_numpy(np.diff(b.q_off[a:e + 1])).to(DEV)
        base = torch.repeat_interleave(x_off_d[a:e], counts)
        nk = torch.repeat_interleave(x_off_d[a + 1:e + 1] - x_off_d[a:e] - 1, counts)
        i = out[q0:q1].long()
        assert bool(torch.all((i >= 0) & (i < nk)))
        zz = z[q0:q1]
        assert bool(torch.all(X_d[base + i] <= zz)) and bool(torch.all(zz < X_d[base + i + 1]))
        del counts, base, nk, i
    pos = np.sort(np.random.default_rng(14).integers(0, int(b.q_off[-1]), 1 << 18))
    zs = z[torch.from_numpy(pos).to(DEV)].cpu().numpy()
    got = out[torch.from_numpy(pos).to(DEV)].cpu().numpy()
    ks = np.searchsorted(b.q_off, pos, side="right") - 1
    ref = np.empty_like(got)
    for k in np.unique(ks):
        sel = ks == k
        ref[sel] = oracle.search(b.array(k), zs[sel])
    _assert_same(got, ref)
