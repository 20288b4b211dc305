"""Seeded synthetic inputs for the interval-search workloads.

This module only draws numbers: it holds none of the search method's
arithmetic, and both the GPU library's tests/benchmarks and the CPU oracle take
their inputs from here.  Every generator is deterministic in its seed.

Shapes follow the paper's test layouts (Sec. 6.1: arrays built from i.i.d.
positive gaps, queries spread over [X_0, X_N)) at the sizes of the workloads
this project measures:

* ``plain_f32_1024``   one f32 array, N = 1024, gaps ~ U(0.5, 1.5), X_0 = 0,
                       10^6 uniform queries plus the adversarial families
                       z = X_i and z = nextafter(X_i, -inf).
* ``sweep``            N in {16, 256, 4096, 65536, 2^20, 2^21}, f32 and f64,
                       gaps ~ U(0.5, 1.5) normalised to [0, 1], queries
                       z = k 2^-p exactly representable and uniform in [0, 1).
* ``clustered``        f64, N + 1 = 2^20 sorted unique draws of exp(N(0, 2));
                       half uniform queries, half X_k (1 + U(-1e-12, 1e-12)).
* ``batched_f32``      10,000 f32 arrays, N_k log-uniform in [8, 65536],
                       offset ~ U(-1e3, 1e3), gaps ~ U(0.5, 1.5), M_k = 64 N_k.
* ``near_limit_array`` small arrays whose smallest gap is about one ulp of the
                       largest key (the feasibility limit of Sec. 4.4), where
                       the choice of H is sensitive to rounding.
* ``batched_mixture``  256 f64 arrays, N_k log-uniform in [2^14, 2^20], each an
                       even mixture of uniform gaps, 8 Gaussian clusters and
                       lognormal tails.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# fixed 64-bit seeds, one per workload
SEED_PLAIN = 0x1506_0862_0000_0001
SEED_SWEEP = 0x1506_0862_0000_0002
SEED_CLUSTERED = 0x1506_0862_0000_0003
SEED_BATCHED = 0x1506_0862_0000_0004
SEED_MIXTURE = 0x1506_0862_0000_0005

SWEEP_N = (16, 256, 4096, 65536, 1 << 20, 1 << 21)
SWEEP_M = 1 << 26


def _rng(seed: int, *stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed & (2**64 - 1), *stream])))


def _dtype(dt) -> np.dtype:
    dt = np.dtype(dt)
    if dt not in (np.dtype(np.float32), np.dtype(np.float64)):
        raise ValueError("dtype must be float32 or float64")
    return dt


def strictly_increasing(x: np.ndarray) -> bool:
    return bool(np.all(x[1:] > x[:-1])) and bool(np.all(np.isfinite(x)))


def prev_float(x, dtype) -> np.ndarray:
    """nextafter(x, -inf) in the given precision."""
    dt = _dtype(dtype)
    return np.nextafter(np.asarray(x, dt), dt.type(-np.inf))


def gap_array(n: int, dtype, rng: np.random.Generator, lo=0.5, hi=1.5, x0=0.0) -> np.ndarray:
    """X_0 = x0, X_{i+1} = X_i + g_i, g_i ~ U(lo, hi); summed in f64, rounded once."""
    g = rng.uniform(lo, hi, size=n)
    x = np.empty(n + 1, np.float64)
    x[0] = x0
    np.cumsum(g, out=x[1:])
    x[1:] += x0
    out = x.astype(_dtype(dtype))
    if not strictly_increasing(out):
        raise RuntimeError("generated array is not strictly increasing after rounding")
    return out


def near_limit_array(dtype, rng: np.random.Generator, q: int = 1, n_fill: int = 0,
                     offset: bool = False) -> np.ndarray:
    """An array at the feasibility limit of Sec. 4.4 (smallest gap about one ulp of the
    largest key): 2..12 consecutive floats ending at a power of two 2^e (e in [-3, 3]),
    q + 1 points at 2^(e-s) (s in [2, 7]) spaced g = U(0.5, 1) times the spacing of the
    run, and n_fill keys evenly spaced in between, each moved by up to a quarter of their
    spacing.  X_0 = 0, or with offset a negative X_0 of up to the low points' magnitude."""
    dt = _dtype(dtype)
    e = int(rng.integers(-3, 4))
    top = dt.type(2.0 ** e)
    run = [top]
    for _ in range(int(rng.integers(q + 1, 12))):
        run.append(np.nextafter(run[-1], dt.type(0)))
    u = np.spacing(run[-1])
    low = dt.type(2.0 ** (e - int(rng.integers(2, 8))))
    g = dt.type(u * rng.uniform(0.5, 1.0))
    pts = [low]
    for _ in range(q):
        pts.append(dt.type(pts[-1] + g))
    a, b = 2.0 * float(low), 0.5 * float(top)
    step = (b - a) / max(n_fill, 1)
    fill = (a + step * (np.arange(n_fill) + 0.5 + rng.uniform(-0.25, 0.25, n_fill))).astype(dt)
    x0 = dt.type(-rng.uniform(0.0, 1.0) * float(low)) if offset else dt.type(0)
    return np.unique(np.concatenate([[x0], pts, fill, run]).astype(dt))


def uniform_queries(x0, xn, m: int, dtype, rng: np.random.Generator) -> np.ndarray:
    """z = x0 + u (xn - x0), u ~ U[0, 1), computed in f64, rounded, kept below xn."""
    dt = _dtype(dtype)
    u = rng.random(m)
    z = (float(x0) + u * (float(xn) - float(x0))).astype(dt)
    top = prev_float(dt.type(xn), dt)
    np.minimum(z, top, out=z)
    np.maximum(z, dt.type(x0), out=z)
    return z


# ----------------------------------------------------------------------------
# one f32 array, N = 1024


@dataclass
class PlainCase:
    X: np.ndarray
    z_uniform: np.ndarray
    z_hits: np.ndarray        # z = X_i, i in [0, N)         -> expected i
    z_below: np.ndarray       # z = nextafter(X_i, -inf), i in [1, N] -> expected i - 1
    z_outside: np.ndarray     # out-of-domain values

    @property
    def N(self) -> int:
        return self.X.size - 1

    @property
    def z_all(self) -> np.ndarray:
        return np.concatenate([self.z_uniform, self.z_hits, self.z_below])


def plain_f32_1024(seed: int = SEED_PLAIN, m: int = 1_000_000, n: int = 1024) -> PlainCase:
    rng = _rng(seed)
    X = gap_array(n, np.float32, rng)
    z = uniform_queries(X[0], X[-1], m, np.float32, rng)
    hits = X[:-1].copy()
    below = prev_float(X[1:], np.float32)
    f32 = np.float32
    outside = np.array([prev_float(X[0], f32), X[-1], np.nextafter(X[-1], f32(np.inf)),
                        f32(-1e30), f32(1e30), f32(np.inf), f32(-np.inf), f32(np.nan),
                        f32(-0.0)], dtype=f32)
    return PlainCase(X, z, hits, below, outside)


# ----------------------------------------------------------------------------
# the N sweep in f32 and f64


def sweep_array(n: int, dtype, seed: int = SEED_SWEEP) -> np.ndarray:
    """S = cumulative sums of U(0.5, 1.5) gaps in f64; X_i = RN(S_i / S_N); X_0 = 0, X_N = 1."""
    dt = _dtype(dtype)
    rng = _rng(seed, n, dt.itemsize)
    g = rng.uniform(0.5, 1.5, size=n)
    s = np.empty(n + 1, np.float64)
    s[0] = 0.0
    np.cumsum(g, out=s[1:])
    x = (s / s[-1]).astype(dt)
    x[-1] = dt.type(1.0)
    if not strictly_increasing(x):
        raise RuntimeError(f"sweep array N={n} {dt} not strictly increasing after rounding")
    return x


def sweep_queries(m: int, dtype, seed: int = SEED_SWEEP, stream: int = 0) -> np.ndarray:
    """z = k 2^-p with k uniform: exact, uniform over [0, 1); p = 24 (f32) or 53 (f64)."""
    dt = _dtype(dtype)
    rng = _rng(seed, 7, dt.itemsize, stream)
    p = 24 if dt == np.float32 else 53
    k = rng.integers(0, 1 << p, size=m, dtype=np.int64)
    return (k.astype(np.float64) * 2.0 ** -p).astype(dt)


def sweep_queries_torch(m: int, dtype, device, seed: int = SEED_SWEEP, stream: int = 0):
    """Device-side variant of sweep_queries with torch's counter-based generator
    (same distribution, different stream of numbers); used where M is large."""
    import torch

    dt = _dtype(dtype)
    g = torch.Generator(device=device)
    g.manual_seed((seed ^ (dt.itemsize << 8) ^ stream) & (2**63 - 1))
    p = 24 if dt == np.float32 else 53
    k = torch.randint(0, 1 << p, (m,), dtype=torch.int64, device=device, generator=g)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    return (k.to(torch.float64) * (2.0 ** -p)).to(tdt)


# ----------------------------------------------------------------------------
# clustered f64 array (lognormal draws)


def clustered_array(n_plus_1: int = 1 << 20, seed: int = SEED_CLUSTERED, sigma: float = 2.0) -> np.ndarray:
    """Sorted unique draws of exp(Normal(0, sigma)), topped up to exactly n_plus_1 values."""
    rng = _rng(seed, 1)
    vals = np.unique(np.exp(rng.normal(0.0, sigma, size=n_plus_1)))
    while vals.size < n_plus_1:
        extra = np.exp(rng.normal(0.0, sigma, size=n_plus_1 - vals.size + 16))
        vals = np.unique(np.concatenate([vals, extra]))
    if vals.size > n_plus_1:
        keep = np.sort(rng.choice(vals.size, size=n_plus_1, replace=False))
        vals = vals[keep]
    assert strictly_increasing(vals)
    return vals.astype(np.float64)


def clustered_queries(X: np.ndarray, m: int, seed: int = SEED_CLUSTERED) -> np.ndarray:
    """Half uniform over [X_0, X_N), half X_k (1 + U(-1e-12, 1e-12)), clamped into [X_0, X_N)."""
    rng = _rng(seed, 2)
    half = m // 2
    zu = uniform_queries(X[0], X[-1], half, np.float64, rng)
    k = rng.integers(0, X.size, size=m - half)
    zc = X[k] * (1.0 + rng.uniform(-1e-12, 1e-12, size=m - half))
    zc = np.clip(zc, X[0], prev_float(X[-1], np.float64))
    z = np.concatenate([zu, zc])
    rng.shuffle(z)
    return z


# ----------------------------------------------------------------------------
# batched ragged workloads


@dataclass
class Batch:
    dtype: np.dtype
    x_off: np.ndarray   # int64[K + 1], offsets into X_packed (array k has x_off[k+1]-x_off[k] values)
    X: np.ndarray       # packed arrays
    q_off: np.ndarray   # int64[K + 1], offsets into z_packed
    z: np.ndarray | None  # packed queries (None when generated on the device)

    @property
    def num_arrays(self) -> int:
        return self.x_off.size - 1

    def array(self, k: int) -> np.ndarray:
        return self.X[self.x_off[k]:self.x_off[k + 1]]

    def queries(self, k: int) -> np.ndarray:
        return self.z[self.q_off[k]:self.q_off[k + 1]]


def log_uniform_int(rng, lo: int, hi: int, size: int) -> np.ndarray:
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=size))).astype(np.int64).clip(lo, hi)


def batched_f32(num_arrays: int = 10_000, n_lo: int = 8, n_hi: int = 65536, q_per_n: int = 64,
                seed: int = SEED_BATCHED, with_queries: bool = True, n_override=None) -> Batch:
    """num_arrays f32 arrays of N_k ~ logU[n_lo, n_hi] gaps U(0.5, 1.5) at offset U(-1e3, 1e3);
    M_k = q_per_n N_k queries uniform in [X_0k, X_Nk)."""
    rng = _rng(seed, 1)
    ns = log_uniform_int(rng, n_lo, n_hi, num_arrays) if n_override is None else np.asarray(n_override, np.int64)
    offs = rng.uniform(-1e3, 1e3, size=ns.size)
    x_off = np.zeros(ns.size + 1, np.int64)
    np.cumsum(ns + 1, out=x_off[1:])
    q_off = np.zeros(ns.size + 1, np.int64)
    np.cumsum(ns * q_per_n, out=q_off[1:])
    X = np.empty(int(x_off[-1]), np.float32)
    for k, n in enumerate(ns):
        X[x_off[k]:x_off[k + 1]] = gap_array(int(n), np.float32, _rng(seed, 2, k), x0=offs[k])
    z = None
    if with_queries:
        z = np.empty(int(q_off[-1]), np.float32)
        for k in range(ns.size):
            xa = X[x_off[k]:x_off[k + 1]]
            z[q_off[k]:q_off[k + 1]] = uniform_queries(xa[0], xa[-1], int(q_off[k + 1] - q_off[k]),
                                                       np.float32, _rng(seed, 3, k))
    return Batch(np.dtype(np.float32), x_off, X, q_off, z)


def mixture_array(n: int, rng: np.random.Generator, length: float = 1.0) -> np.ndarray:
    """n + 1 sorted unique f64 values: one third from a uniform-gap walk over [0, L),
    one third from 8 Gaussian clusters (centres ~ U[0, L), sigma = 1e-4 L),
    one third from L exp(N(0, 2)) lognormal tails."""
    target = n + 1
    parts = []
    a = target // 3
    b = target // 3
    c = target - a - b
    g = rng.uniform(0.5, 1.5, size=a)
    walk = np.cumsum(g)
    parts.append(walk / walk[-1] * length * (1 - 1e-9))
    centres = rng.uniform(0.0, length, size=8)
    which = rng.integers(0, 8, size=b)
    parts.append(centres[which] + rng.normal(0.0, 1e-4 * length, size=b))
    parts.append(length * np.exp(rng.normal(0.0, 2.0, size=c)))
    vals = np.unique(np.concatenate(parts))
    while vals.size < target:
        extra = rng.uniform(0.0, length, size=target - vals.size)
        vals = np.unique(np.concatenate([vals, extra]))
    if vals.size > target:
        keep = np.sort(rng.choice(vals.size, size=target, replace=False))
        vals = vals[keep]
    assert strictly_increasing(vals)
    return vals


def batched_mixture(num_arrays: int = 256, n_lo: int = 1 << 14, n_hi: int = 1 << 20,
                    total_queries: int = 1 << 28, seed: int = SEED_MIXTURE,
                    with_queries: bool = True) -> Batch:
    """num_arrays f64 mixture arrays; queries proportional to N_k, split 70 % uniform,
    20 % exact hits X_i (i < N), 10 % nextafter(X_i, -inf) (i >= 1)."""
    rng = _rng(seed, 1)
    ns = log_uniform_int(rng, n_lo, n_hi, num_arrays)
    x_off = np.zeros(ns.size + 1, np.int64)
    np.cumsum(ns + 1, out=x_off[1:])
    share = ns / ns.sum()
    mk = np.floor(share * total_queries).astype(np.int64)
    mk[-1] += total_queries - mk.sum()
    q_off = np.zeros(ns.size + 1, np.int64)
    np.cumsum(mk, out=q_off[1:])
    X = np.empty(int(x_off[-1]), np.float64)
    for k, n in enumerate(ns):
        X[x_off[k]:x_off[k + 1]] = mixture_array(int(n), _rng(seed, 2, k))
    z = None
    if with_queries:
        z = np.empty(int(q_off[-1]), np.float64)
        for k in range(ns.size):
            xa = X[x_off[k]:x_off[k + 1]]
            z[q_off[k]:q_off[k + 1]] = mixture_queries(xa, int(mk[k]), _rng(seed, 3, k))
    return Batch(np.dtype(np.float64), x_off, X, q_off, z)


def mixture_queries(X: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    n = X.size - 1
    mu = int(round(0.7 * m))
    mh = int(round(0.2 * m))
    mb = m - mu - mh
    zu = uniform_queries(X[0], X[-1], mu, X.dtype, rng)
    zh = X[rng.integers(0, n, size=mh)]
    zb = prev_float(X[rng.integers(1, n + 1, size=mb)], X.dtype)
    z = np.concatenate([zu, zh, zb]).astype(X.dtype)
    rng.shuffle(z)
    return z


def batched_queries_torch(batch: Batch, device, seed: int = SEED_BATCHED, chunk_arrays: int = 256):
    """Uniform queries per array, z ~ U[X_0k, X_Nk), generated on the device with
    torch's counter-based generator: z = X_0k + u (X_Nk - X_0k) in f64, rounded to the
    batch dtype and kept below X_Nk.  Returns the packed query tensor."""
    import torch

    tdt = torch.float32 if batch.dtype == np.float32 else torch.float64
    total = int(batch.q_off[-1])
    z = torch.empty(total, dtype=tdt, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed & (2**63 - 1))
    K = batch.num_arrays
    lo_all = batch.X[batch.x_off[:-1]].astype(np.float64)
    hi_all = batch.X[batch.x_off[1:] - 1].astype(np.float64)
    hi_below = prev_float(batch.X[batch.x_off[1:] - 1], batch.dtype).astype(np.float64)
    for a in range(0, K, chunk_arrays):
        b = min(K, a + chunk_arrays)
        q0, q1 = int(batch.q_off[a]), int(batch.q_off[b])
        if q1 == q0:
            continue
        counts = torch.from_numpy(np.diff(batch.q_off[a:b + 1])).to(device)
        lo = torch.repeat_interleave(torch.from_numpy(lo_all[a:b]).to(device), counts)
        hi = torch.repeat_interleave(torch.from_numpy(hi_all[a:b]).to(device), counts)
        top = torch.repeat_interleave(torch.from_numpy(hi_below[a:b]).to(device), counts)
        u = torch.rand(q1 - q0, dtype=torch.float64, device=device, generator=g)
        v = (lo + u * (hi - lo)).to(tdt)
        z[q0:q1] = torch.minimum(torch.maximum(v, lo.to(tdt)), top.to(tdt))
        del lo, hi, top, u, v
    return z


def batched_mixture_queries_torch(batch: Batch, device, seed: int = SEED_MIXTURE, chunk_arrays: int = 16):
    """Device-side queries of the mixture workload: per array 70 % uniform in [X_0, X_N),
    20 % exact hits X_i (i < N), 10 % nextafter(X_i, -inf) (i >= 1), shuffled within the array."""
    import torch

    tdt = torch.float32 if batch.dtype == np.float32 else torch.float64
    total = int(batch.q_off[-1])
    z = torch.empty(total, dtype=tdt, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed & (2**63 - 1))
    X_d = torch.from_numpy(batch.X).to(device)
    for k in range(batch.num_arrays):
        q0, q1 = int(batch.q_off[k]), int(batch.q_off[k + 1])
        m = q1 - q0
        if m == 0:
            continue
        x0, x1 = int(batch.x_off[k]), int(batch.x_off[k + 1])
        n = x1 - x0 - 1
        mu = int(round(0.7 * m))
        mh = int(round(0.2 * m))
        mb = m - mu - mh
        lo, hi = float(batch.X[x0]), float(batch.X[x1 - 1])
        u = torch.rand(mu, dtype=torch.float64, device=device, generator=g)
        zu = (lo + u * (hi - lo)).to(tdt)
        top = torch.nextafter(X_d[x1 - 1:x1], torch.tensor([-np.inf], dtype=tdt, device=device))
        zu = torch.minimum(torch.maximum(zu, X_d[x0:x0 + 1]), top)
        ih = torch.randint(0, n, (mh,), device=device, generator=g) + x0
        ib = torch.randint(1, n + 1, (mb,), device=device, generator=g) + x0
        zb = torch.nextafter(X_d[ib], torch.full((mb,), -np.inf, dtype=tdt, device=device))
        zz = torch.cat([zu, X_d[ih], zb])
        perm = torch.randperm(m, device=device, generator=g)
        z[q0:q1] = zz[perm]
    return z
