"""Pins of the oracle's Eytzinger layout and search (Sec. 3.4, the cache-friendly
binary search) against facts fixed by the paper and by mathematics.

CPU only.  The layout is the padded array (X, then copies of X_N up to
2^L - 1 values) in breadth-first order of the complete binary search tree.
Pinned by: hand-built layouts of a perfect and an imperfect tree, an
independent in-order walk that must give back the padded array, brute force on
tiny arrays, the library's searchsorted, exhaustive enumeration of a float
span, and the extra level of the height printed in the section.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import _float_span, _queries_for, _random_tiny


def _inorder(Y, L):
    """Iterative in-order walk of nodes 1 .. 2^L - 1 (children 2k, 2k + 1)."""
    nodes = (1 << L) - 1
    out, stack, k = [], [], 1
    while stack or k <= nodes:
        while k <= nodes:
            stack.append(k)
            k = 2 * k
        k = stack.pop()
        out.append(Y[k])
        k = 2 * k + 1
    return np.array(out, Y.dtype)


def _padded(X, L):
    return np.concatenate([X, np.full((1 << L) - 1 - X.size, X[-1], X.dtype)])


def test_hand_built_layouts():
    X = np.array([1.0, 2.0, 3.0], np.float64)  # N = 2: L = 2, a perfect tree of 3 nodes
    st, Y = oracle.eytzinger_layout(X)
    assert st == oracle.OK and oracle.eytzinger_levels(2) == 2
    assert list(Y[1:]) == [2.0, 1.0, 3.0]
    X = np.arange(7, dtype=np.float32)  # N = 6: L = 3, 7 nodes, no padding
    st, Y = oracle.eytzinger_layout(X)
    assert list(Y[1:]) == [3, 1, 5, 0, 2, 4, 6]
    X = np.arange(8, dtype=np.float32)  # N = 7: L = 4, 15 nodes, 7 copies of X_7 = 7
    st, Y = oracle.eytzinger_layout(X)
    assert oracle.eytzinger_levels(7) == 4
    assert list(Y[1:]) == [7, 3, 7, 1, 5, 7, 7, 0, 2, 4, 6, 7, 7, 7, 7]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_layout_is_the_padded_array_in_tree_order(dt):
    rng = np.random.default_rng(1)
    for n in list(range(1, 40)) + [255, 256, 1000, 4095, 4096]:
        X = _random_tiny(rng, n, dt)
        L = oracle.eytzinger_levels(n)
        assert (1 << L) - 1 >= n + 1 > (1 << (L - 1)) - 1
        st, Y = oracle.eytzinger_layout(X)
        assert st == oracle.OK
        assert np.array_equal(_inorder(Y, L), _padded(X, L))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_search_matches_brute_force_and_library(dt):
    rng = np.random.default_rng(2)
    for n in list(range(1, 70)) + [1023, 1024, 1025]:
        X = _random_tiny(rng, n, dt)
        L = oracle.eytzinger_levels(n)
        st, Y = oracle.eytzinger_layout(X)
        z = _queries_for(X, rng, m=500)
        got = oracle.eytzinger_search(Y, n, L, z)
        assert np.array_equal(got, oracle.brute(X, z) if n < 100 else oracle.search(X, z)), n
    X = W.sweep_array(65536, dt)
    st, Y = oracle.eytzinger_layout(X)
    z = W.sweep_queries(200_000, dt)
    got = oracle.eytzinger_search(Y, 65536, oracle.eytzinger_levels(65536), z)
    assert np.array_equal(got, (np.searchsorted(X, z, side="right") - 1).astype(np.int32))


def test_printed_height_with_an_extra_level():
    """The section's L = 1 + floor(log2(2 + N)) is one level more than needed when N + 2 is a
    power of two; the extra padding leaves every result unchanged."""
    rng = np.random.default_rng(3)
    for n in (2, 6, 14, 30, 62, 126):
        X = _random_tiny(rng, n, np.float64)
        Lp = 1 + int(np.floor(np.log2(2 + n)))
        assert Lp == oracle.eytzinger_levels(n) + 1
        st, Y = oracle.eytzinger_layout(X, Lp)
        z = _queries_for(X, rng, m=500)
        assert np.array_equal(oracle.eytzinger_search(Y, n, Lp, z), oracle.brute(X, z))


def test_exhaustive_f32_span():
    dt = np.float32
    span = _float_span(dt(0.75), 1 << 20, dt)
    rng = np.random.default_rng(4)
    pick = np.sort(rng.choice(span.size - 2, size=500, replace=False)) + 1
    X = np.concatenate([[span[0]], span[pick], [span[-1]]]).astype(dt)
    n = X.size - 1
    st, Y = oracle.eytzinger_layout(X)
    z = span[:-1]
    got = oracle.eytzinger_search(Y, n, oracle.eytzinger_levels(n), z)
    assert np.array_equal(got, (np.searchsorted(X, z, side="right") - 1).astype(np.int32))


def test_layout_rejects_too_few_levels():
    X = np.arange(8, dtype=np.float32)
    assert oracle.eytzinger_layout(X, 3)[0] == oracle.ERR_ARG
