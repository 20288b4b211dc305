"""ds_search_batched_noalloc (the batched build + search on the library's fixed
per-GPU scratch array) against ds_search_batched on the caller's workspace:
identical indices, call after call, the later calls on smaller batches (the
scratch keeps the previous call's contents), and both equal to the oracle."""
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


def _oracle_batch(b):
    ref = np.empty(b.z.size, np.int32)
    for k in range(b.x_off.size - 1):
        q0, q1 = b.q_off[k], b.q_off[k + 1]
        if q1 == q0:
            continue
        xa = b.X[b.x_off[k]:b.x_off[k + 1]]
        ref[q0:q1] = -1 if xa.size == 0 else oracle.search(xa, b.z[q0:q1])
    return ref


def _mixture_batch(ns, m_each, seed):
    rng = np.random.default_rng(seed)
    arrays = [W.mixture_array(int(n), rng) for n in ns]
    zs = [W.mixture_queries(a, m_each, rng) for a in arrays]
    x_off = np.concatenate([[0], np.cumsum([a.size for a in arrays])]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum([q.size for q in zs])]).astype(np.int64)
    return W.Batch(np.dtype(np.float64), x_off, np.concatenate(arrays), q_off, np.concatenate(zs))


def _check(ds, b, **kw):
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z), **kw)
    ref = bt.run().clone()
    got = torch.full_like(ref, -7)
    bt.run_noalloc(out=got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    want = _oracle_batch(b)
    g = got.cpu().numpy()
    if not np.array_equal(g, want):
        bad = np.flatnonzero(g != want)
        raise AssertionError(f"{bad.size} of {want.size} differ from the oracle; first at {bad[:5]}")


def test_noalloc_equals_workspace_entry_point(ds):
    print("noalloc: 300 f32 arrays", flush=True)
    _check(ds, W.batched_f32(num_arrays=300, n_lo=8, n_hi=8192, q_per_n=16, seed=31))
    print("noalloc: 40 f32 arrays (smaller, after the larger call)", flush=True)
    _check(ds, W.batched_f32(num_arrays=40, n_lo=8, n_hi=2048, q_per_n=8, seed=32), form="fma")
    print("noalloc: 4 f64 mixture arrays, learned models", flush=True)
    _check(ds, _mixture_batch((3000, 9000, 20000, 500), 20_000, 33), learn_segments=512, learn_steps=8,
           direct_cap_bytes=64)
    print("noalloc: 3 f64 mixture arrays, smaller", flush=True)
    _check(ds, _mixture_batch((700, 4000, 60), 5_000, 34), learn_segments=256, learn_steps=4)


def test_noalloc_rejects_batches_over_the_scratch(ds):
    """A batch whose fixed workspace alone exceeds the scratch array is refused on the host
    (nothing is launched)."""
    b = W.batched_f32(num_arrays=4, n_lo=8, n_hi=64, q_per_n=4, seed=35)
    too_many = ds.NOALLOC_SCRATCH_BYTES // 2 + 1  # 2-byte codes per value alone exceed it
    assert ds.batch_workspace_bytes(4, too_many, 0, 0) > ds.NOALLOC_SCRATCH_BYTES
    bt = ds.Batch(_dev(b.x_off), _dev(b.X), _dev(b.q_off), _dev(b.z), total_x=too_many, table_budget_entries=0)
    with pytest.raises(ds.DsError) as e:
        bt.run_noalloc()
    assert e.value.status == ds.ERR_SCRATCH_CAP
