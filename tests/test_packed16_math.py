"""CPU pins of the two facts the capped 16-bit mode (APSP_FLAG_PACKED16)
rests on, checked against the oracle on small graphs:

1. Capping commutes with the semiring: Floyd-Warshall run in arithmetic
   capped at c (every sum min(a + b, c)) gives min(true distance, c).
2. The int32 redo is exact: the closure of any matrix M with
   closure(W) <= M <= W (entrywise) is closure(W).

The capped Floyd-Warshall here is written in the test, from Eq. 1 with the
capped addition; the oracle supplies the true closure.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

INF = 1 << 30


def capped_fw(W, cap):
    X = np.minimum(W.astype(np.int64), cap)
    for k in range(X.shape[0]):
        X = np.minimum(X, np.minimum(X[:, k:k + 1] + X[k:k + 1, :], cap))
    return X


def random_graph(rng, n, p, hi):
    W = np.where(rng.random((n, n)) < p, rng.integers(0, hi + 1, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


@settings(max_examples=60, deadline=None)
@given(n=st.integers(1, 24), p=st.floats(0.0, 1.0), hi=st.sampled_from([3, 50, 1000, 40000]),
       cap=st.sampled_from([1, 7, 100, 0x39FF, 0x7FFF]), seed=st.integers(0, 2**31))
def test_capping_commutes_with_the_closure(n, p, hi, cap, seed):
    W = random_graph(np.random.default_rng(seed), n, p, hi)
    true = oracle.fw_i32(W).astype(np.int64)
    np.testing.assert_array_equal(capped_fw(W, cap), np.minimum(true, cap))


@settings(max_examples=60, deadline=None)
@given(n=st.integers(1, 24), p=st.floats(0.0, 1.0), hi=st.sampled_from([3, 1000, 40000]),
       seed=st.integers(0, 2**31))
def test_redo_from_any_matrix_between_closure_and_input(n, p, hi, seed):
    rng = np.random.default_rng(seed)
    W = random_graph(rng, n, p, hi)
    true = oracle.fw_i32(W)
    # M: a random point between closure(W) and W, entrywise
    lo, up = true.astype(np.int64), W.astype(np.int64)
    M = (lo + (rng.random(W.shape) * (up - lo + 1)).astype(np.int64)).clip(lo, up).astype(np.int32)
    np.testing.assert_array_equal(oracle.fw_i32(M), true)


def test_a_capped_entry_hides_a_finite_distance():
    # why the redo is needed: a path of length 3 * 9000 reads as "no path" under the cap
    W = np.full((4, 4), INF, np.int32)
    np.fill_diagonal(W, 0)
    W[0, 1] = W[1, 2] = W[2, 3] = 9000
    true = oracle.fw_i32(W)
    assert true[0, 3] == 27000
    assert capped_fw(W, 0x39FF)[0, 3] == 0x39FF


def test_binary16_patterns_order_like_integers():
    # the packed products take integer minima with a binary16 minimum on the
    # bit patterns: staged values are min(v, cap) + 0x400, sums carry 0x800
    cap, off = 0x39FF, 0x400
    pats = np.arange(off, 2 * (cap + off) + 1, dtype=np.uint16)
    vals = pats.view(np.float16).astype(np.float64)
    assert np.all(np.isfinite(vals)) and np.all(vals > 0)
    assert np.all(np.diff(vals) > 0)                      # strictly increasing with the pattern
    assert 2 * (cap + off) <= 0x7BFF                      # largest sum: the largest finite binary16
    assert 2 * (cap + off) < 1 << 16                      # no carry into the next 16-bit lane
