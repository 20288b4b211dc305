"""Pins of the fp64 router reference (oracle/mlp.py): finite differences and
closed forms.  CPU only."""
import numpy as np

from oracle import mlp


def _params(rng, spread=True):
    p = np.empty(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = [None] * 6
    o = 0
    w1 = rng.uniform(2, 6, 32)
    c = rng.uniform(0.1, 0.9, 32)
    p[0:32] = w1
    p[32:64] = 0.5 - w1 * c
    W2 = rng.uniform(0, 2.0 / 32, (32, 32))
    p[64:64 + 1024] = W2.reshape(-1)
    p[1088:1120] = 0.5 - 0.5 * W2.sum(1) + rng.uniform(-0.1, 0.1, 32)
    p[1120:1152] = rng.uniform(0, 1.0 / 16, 32)
    p[1152] = rng.uniform(-0.1, 0.1)
    return p


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(rng)
    u = rng.uniform(0, 1, 200)
    t = np.sort(rng.uniform(0, 1, 200))
    _, g = mlp.grad(p, u, t)
    idx = list(range(0, 64)) + list(rng.choice(np.arange(64, 1088), 60, replace=False)) + list(range(1088, 1153))
    num = mlp.numeric_grad(p, u, t, idx, eps=1e-7)
    # kinks of clamp are measure-zero; with these samples no unit sits within eps of 0 or 1
    np.testing.assert_allclose(g[idx], num, rtol=1e-5, atol=1e-9)


def test_closed_form_constant_network():
    """W2 = 0: every layer-2 unit outputs clamp(b2), y is a constant, layer 1
    gets no gradient, and the other gradients have closed forms."""
    rng = np.random.default_rng(1)
    p = _params(rng)
    p[64:1088] = 0.0
    b2 = np.linspace(-0.5, 1.5, 32)
    p[1088:1120] = b2
    u = rng.uniform(0, 1, 50)
    t = rng.uniform(0, 1, 50)
    h2 = np.clip(b2, 0, 1)
    W3 = p[1120:1152]
    y = h2 @ W3 + p[1152]
    loss, g = mlp.grad(p, u, t)
    r = 2 * np.mean(y - t)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-12
    np.testing.assert_allclose(g[1120:1152], r * h2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(g[1152], r, rtol=1e-12)
    inside = (b2 > 0) & (b2 < 1)
    np.testing.assert_allclose(g[1088:1120], np.where(inside, r * W3, 0.0), rtol=1e-12, atol=1e-15)
    assert np.all(g[0:64] == 0)
    dy = 2 * (y - t) / t.size
    h1 = np.clip(np.outer(u, p[0:32]) + p[32:64], 0, 1)
    gW2 = np.outer(np.where(inside, W3, 0.0), dy @ h1)
    np.testing.assert_allclose(g[64:1088], gW2.reshape(-1), rtol=1e-12, atol=1e-15)


def test_monotone_with_nonnegative_weights():
    rng = np.random.default_rng(2)
    p = _params(rng)
    u = np.sort(rng.uniform(-0.2, 1.2, 10000))
    y, _ = mlp.forward(p, u)
    assert np.all(np.diff(y) >= 0)
    # a negative weight can break it (the property needs the projection)
    p2 = p.copy()
    p2[1120:1152] = -p2[1120:1152]
    y2, _ = mlp.forward(p2, u)
    assert np.any(np.diff(y2) < 0)
