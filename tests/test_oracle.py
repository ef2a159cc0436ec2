"""Pins for the CPU oracle (no GPU).

The paper prints no numeric worked example, so the oracle is pinned to things
other than itself: hand-worked fixtures (tests/golden/), exhaustive simple-path
enumeration on tiny graphs, Dijkstra (an independent algorithm), BFS on unit
weights, closed forms and invariants.  The last block plants plausible
mistakes in copies of the oracle's recurrences and checks that the same pins
catch every one of them.
"""
import itertools

import numpy as np
import pytest

import golden_io

INF = 1 << 30


def rand_graph(rng, n, p, lo, hi, zero_frac=0.0):
    W = np.full((n, n), INF, dtype=np.int32)
    mask = rng.random((n, n)) < p
    w = rng.integers(lo, hi + 1, size=(n, n))
    if zero_frac:
        w[rng.random((n, n)) < zero_frac] = 0
    W[mask] = w[mask]
    np.fill_diagonal(W, 0)
    return W


# ---------------------------------------------------------------------------
# Floyd-Warshall (Sec. 2, Eq. 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", golden_io.fw_fixtures())
def test_fw_golden(oracle, name):
    g = golden_io.load(name)
    np.testing.assert_array_equal(oracle.fw_i32(g["W"]), g["D"])


@pytest.mark.parametrize("name", [f for f in golden_io.fw_fixtures() if "saturate" not in f])
def test_fw_f64_golden(oracle, name):
    g = golden_io.load(name)
    W = g["W"].astype(np.float64)
    W[g["W"] >= INF] = np.inf
    D = g["D"].astype(np.float64)
    D[g["D"] >= INF] = np.inf
    np.testing.assert_array_equal(oracle.fw_f64(W), D)


def test_fw_vs_bruteforce_int(oracle):
    rng = np.random.default_rng(11)
    for trial in range(150):
        n = int(rng.integers(1, 8))
        p = float(rng.choice([0.2, 0.5, 0.9]))
        hi = int(rng.choice([10, 1000, 700_000_000]))   # last one exercises saturation
        W = rand_graph(rng, n, p, 0 if trial % 3 == 0 else 1, hi, zero_frac=0.1 if trial % 5 == 0 else 0)
        ref = np.array(oracle.brute_apsp(W.tolist()), dtype=np.int64)
        np.testing.assert_array_equal(oracle.fw_i32(W), ref, err_msg=f"trial {trial}")


def restricted_bruteforce(W, k):
    """Shortest i -> j distance over simple paths whose intermediate vertices
    all lie below k (enumerated; tiny n), saturated at INF."""
    n = len(W)
    out = np.full((n, n), INF, dtype=np.int64)
    for s in range(n):
        out[s, s] = 0

        def dfs(u, dist, seen):
            for v in range(n):
                if v in seen or W[u][v] >= INF:
                    continue
                nd = dist + int(W[u][v])
                if nd < out[s, v]:
                    out[s, v] = min(nd, INF)
                if v < k:                       # only vertices below k may be passed through
                    dfs(v, nd, seen | {v})

        dfs(s, 0, {s})
    return out


def test_fw_steps_restricted_intermediates(oracle):
    """After passes 0 .. k-1 of Eq. 1, D holds the shortest distances over
    paths with every intermediate vertex below k (brute force); the passes
    compose (0..a then a..n equals the full triple loop)."""
    rng = np.random.default_rng(13)
    for trial in range(60):
        n = int(rng.integers(1, 8))
        W = rand_graph(rng, n, float(rng.choice([0.3, 0.6])), 1, int(rng.choice([9, 1000])))
        for k in range(n + 1):
            np.testing.assert_array_equal(oracle.fw_i32_steps(W, 0, k), restricted_bruteforce(W.tolist(), k),
                                          err_msg=f"trial {trial} k={k}")
    W = rand_graph(rng, 90, 0.05, 1, 100)
    for a in (0, 1, 37, 90):
        np.testing.assert_array_equal(oracle.fw_i32_steps(oracle.fw_i32_steps(W, 0, a), a, 90, threads=3),
                                      oracle.fw_i32(W))


def test_fw_f64_vs_bruteforce(oracle):
    rng = np.random.default_rng(12)
    for trial in range(100):
        n = int(rng.integers(1, 8))
        W = np.where(rng.random((n, n)) < 0.5, rng.uniform(0.1, 10.0, (n, n)), np.inf)
        np.fill_diagonal(W, 0.0)
        ref = np.array(oracle.brute_apsp(W.tolist(), inf=np.inf, saturate=False), dtype=np.float64)
        got = oracle.fw_f64(W)
        np.testing.assert_allclose(got, ref, rtol=1e-12)
        assert np.array_equal(np.isinf(got), np.isinf(ref))


def test_fw_vs_dijkstra_int(oracle):
    rng = np.random.default_rng(13)
    for n, p in [(60, 0.05), (97, 0.1), (150, 0.02), (128, 0.5)]:
        W = rand_graph(rng, n, p, 1, 1000)
        np.testing.assert_array_equal(oracle.fw_i32(W, threads=4),
                                      oracle.dijkstra_i32(W, np.arange(n)))


def test_fw_f64_vs_dijkstra_f64(oracle):
    rng = np.random.default_rng(14)
    n = 120
    W = np.where(rng.random((n, n)) < 0.05, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    D = oracle.fw_f64(W.astype(np.float64))
    R = oracle.dijkstra_f64(W, np.arange(n))
    assert np.array_equal(np.isinf(D), np.isinf(R))
    fin = np.isfinite(R)
    np.testing.assert_allclose(D[fin], R[fin], rtol=1e-12)


def test_fw_unit_weights_is_bfs(oracle):
    rng = np.random.default_rng(15)
    n = 40
    adj = rng.random((n, n)) < 0.06
    np.fill_diagonal(adj, False)
    W = np.where(adj, 1, INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    hops = oracle.bfs_hops(adj.tolist())
    ref = np.array([[INF if h is None else h for h in row] for row in hops], dtype=np.int64)
    np.testing.assert_array_equal(oracle.fw_i32(W), ref)


def test_fw_closed_forms(oracle):
    # no edges: nothing changes
    W = np.full((5, 5), INF, dtype=np.int32)
    np.fill_diagonal(W, 0)
    np.testing.assert_array_equal(oracle.fw_i32(W), W)
    # n = 1 and n = 0
    np.testing.assert_array_equal(oracle.fw_i32(np.zeros((1, 1), np.int32)), [[0]])
    assert oracle.fw_i32(np.zeros((0, 0), np.int32)).shape == (0, 0)
    # directed path 0->1->...->n-1: prefix sums above the diagonal, INF below
    n = 9
    w = np.arange(1, n, dtype=np.int64) * 7
    W = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(W, 0)
    for i in range(n - 1):
        W[i, i + 1] = w[i]
    ref = np.full((n, n), INF, dtype=np.int64)
    pref = np.concatenate([[0], np.cumsum(w)])
    for i in range(n):
        for j in range(i, n):
            ref[i, j] = pref[j] - pref[i]
    np.testing.assert_array_equal(oracle.fw_i32(W), ref)
    # complete graph with equal weights: every off-diagonal distance is w
    W = np.full((7, 7), 13, dtype=np.int32)
    np.fill_diagonal(W, 0)
    np.testing.assert_array_equal(oracle.fw_i32(W), W)


def test_fw_invariants(oracle):
    rng = np.random.default_rng(16)
    n = 70
    W = rand_graph(rng, n, 0.08, 1, 100)
    D = oracle.fw_i32(W).astype(np.int64)
    assert (np.diag(D) == 0).all()
    assert (D <= W).all()
    # triangle inequality for every k (saturating)
    tri = np.minimum(D[:, :, None] + D[None, :, :], INF).min(axis=1)
    assert (D <= tri).all()
    # idempotence: distances are already closed
    np.testing.assert_array_equal(oracle.fw_i32(D.astype(np.int32)), D)
    # symmetric input gives symmetric output
    S = np.minimum(W, W.T)
    DS = oracle.fw_i32(S)
    np.testing.assert_array_equal(DS, DS.T)


# ---------------------------------------------------------------------------
# min-plus product (Sec. 3, Eq. 2)
# ---------------------------------------------------------------------------

def test_minplus_golden(oracle):
    g = golden_io.load("minplus_2x3x2.txt")
    np.testing.assert_array_equal(oracle.minplus_i32(g["A"], g["B"], g["C"]), g["OUT"])


def _minplus_loops(A, B, C, sat):
    m, k = A.shape
    n = B.shape[1]
    out = C.astype(object).copy()
    for i in range(m):
        for j in range(n):
            for t in range(k):
                v = int(A[i, t]) + int(B[t, j]) if sat else float(A[i, t]) + float(B[t, j])
                if sat:
                    v = min(v, INF)
                out[i, j] = min(out[i, j], v)
    return out


def test_minplus_vs_loops_int(oracle):
    rng = np.random.default_rng(21)
    for m, k, n in [(1, 1, 1), (3, 5, 2), (7, 1, 9), (6, 11, 4), (0, 3, 2), (3, 0, 4)]:
        A = np.where(rng.random((m, k)) < 0.7, rng.integers(0, INF + 1, (m, k)), INF).astype(np.int32)
        B = np.where(rng.random((k, n)) < 0.7, rng.integers(0, INF + 1, (k, n)), INF).astype(np.int32)
        C = rng.integers(0, INF + 1, (m, n)).astype(np.int32)
        ref = _minplus_loops(A, B, C, True).astype(np.int64)
        np.testing.assert_array_equal(oracle.minplus_i32(A, B, C), ref)


def test_minplus_f32_single_rounding(oracle):
    # each term is one binary32 addition: fl32(a + b) == float32(double(a) + double(b))
    # (the exact sum of two binary32 values in this range fits in a double)
    rng = np.random.default_rng(22)
    A = rng.uniform(0.1, 10.0, (1, 4000)).astype(np.float32)
    B = rng.uniform(0.1, 10.0, (4000, 1)).astype(np.float32)
    for t in range(4000):
        got = oracle.minplus_f32(A[:, t:t + 1], B[t:t + 1, :])[0, 0]
        ref = np.float32(np.float64(A[0, t]) + np.float64(B[t, 0]))
        assert got == ref
    # and the full product equals the exact per-term rounding, minimised
    A = rng.uniform(0.1, 10.0, (5, 13)).astype(np.float32)
    B = rng.uniform(0.1, 10.0, (13, 6)).astype(np.float32)
    ref = (A.astype(np.float64)[:, :, None] + B.astype(np.float64)[None, :, :]).astype(np.float32).min(axis=1)
    np.testing.assert_array_equal(oracle.minplus_f32(A, B), ref)


def test_minplus_identity_and_associativity(oracle):
    rng = np.random.default_rng(23)
    n = 12
    I = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(I, 0)
    A = rng.integers(0, 1000, (7, n)).astype(np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(A, I), A)
    B = rng.integers(0, 1000, (n, 5)).astype(np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(I, B), B)
    X = rng.integers(0, 1000, (4, 6)).astype(np.int32)
    Y = rng.integers(0, 1000, (6, 8)).astype(np.int32)
    Z = rng.integers(0, 1000, (8, 3)).astype(np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(oracle.minplus_i32(X, Y), Z),
                                  oracle.minplus_i32(X, oracle.minplus_i32(Y, Z)))
    # K = 0 leaves C unchanged
    C = rng.integers(0, INF, (3, 4)).astype(np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(np.zeros((3, 0), np.int32), np.zeros((0, 4), np.int32), C), C)


def test_minplus_saturation(oracle):
    A = np.array([[INF, INF - 1, 1]], dtype=np.int32)
    B = np.array([[INF], [5], [INF]], dtype=np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(A, B), [[INF]])
    B = np.array([[0], [0], [INF - 2]], dtype=np.int32)
    np.testing.assert_array_equal(oracle.minplus_i32(A, B), [[INF - 1]])


def test_fw_is_iterated_minplus_closure(oracle):
    # min-plus squaring to a fixpoint (Sec. 3.2) reaches the FW result
    rng = np.random.default_rng(24)
    W = rand_graph(rng, 40, 0.07, 1, 50)
    D = W.copy()
    for _ in range(10):
        nxt = oracle.minplus_i32(D, D, D)
        if np.array_equal(nxt, D):
            break
        D = nxt
    np.testing.assert_array_equal(D, oracle.fw_i32(W))


# ---------------------------------------------------------------------------
# Dijkstra and the certificate
# ---------------------------------------------------------------------------

def test_dijkstra_vs_bruteforce(oracle):
    rng = np.random.default_rng(31)
    for _ in range(40):
        n = int(rng.integers(1, 8))
        W = rand_graph(rng, n, 0.5, 0, 20)
        ref = np.array(oracle.brute_apsp(W.tolist()), dtype=np.int64)
        np.testing.assert_array_equal(oracle.dijkstra_i32(W, np.arange(n)), ref)


def test_certificate(oracle):
    rng = np.random.default_rng(32)
    n = 80
    W = rand_graph(rng, n, 0.06, 1, 100)
    D = oracle.fw_i32(W)
    assert oracle.certificate_i32(W, D) == 0
    fin = np.argwhere((D < INF) & ~np.eye(n, dtype=bool))
    i, j = fin[len(fin) // 2]
    low = D.copy(); low[i, j] -= 1            # no tight edge any more
    assert oracle.certificate_i32(W, low) > 0
    high = D.copy(); high[i, j] += 1          # some edge now gives a shorter path
    assert oracle.certificate_i32(W, high) > 0
    diag = D.copy(); diag[3, 3] = 1
    assert oracle.certificate_i32(W, diag) > 0
    unreach = np.argwhere(D >= INF)
    if len(unreach):
        a, b = unreach[0]
        fake = D.copy(); fake[a, b] = 10**6   # claims a path that does not exist
        assert oracle.certificate_i32(W, fake) > 0


# ---------------------------------------------------------------------------
# planted mistakes: each mutant of the recurrences must fail some pin
# ---------------------------------------------------------------------------

def _fw_mutant(W, kind):
    D = W.astype(np.int64).copy()
    n = D.shape[0]
    ks = range(n - 1) if kind == "off_by_one" else range(n)
    if kind == "k_innermost":
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    D[i, j] = min(D[i, j], min(D[i, k] + D[k, j], INF))
        return D
    for k in ks:
        for i in range(n):
            for j in range(n):
                if kind == "transposed":
                    via = D[k, i] + D[j, k]
                elif kind == "no_saturation":
                    s = int(D[i, k] + D[k, j]) & 0xFFFFFFFF      # int32 wrap-around
                    D[i, j] = min(D[i, j], s - 2**32 if s >= 2**31 else s)
                    continue
                elif kind == "dropped_min":
                    via = D[i, k] + D[k, j]
                    D[i, j] = min(via, INF) if i != j else 0
                    continue
                else:
                    via = D[i, k] + D[k, j]
                D[i, j] = min(D[i, j], min(via, INF))
    return D


def _fw_pins_pass(fw):
    for name in golden_io.fw_fixtures():
        g = golden_io.load(name)
        if not np.array_equal(fw(g["W"]), g["D"]):
            return False
    rng = np.random.default_rng(41)
    for _ in range(60):
        n = int(rng.integers(2, 7))
        W = rand_graph(rng, n, 0.5, 1, 700_000_000 if _ % 4 == 0 else 20)
        if not np.array_equal(fw(W), np.array(golden_io_brute(W))):
            return False
    return True


def golden_io_brute(W):
    import oracle
    return oracle.brute_apsp(W.tolist())


def test_oracle_fw_passes_pins(oracle):
    assert _fw_pins_pass(oracle.fw_i32)


@pytest.mark.parametrize("kind", ["transposed", "k_innermost", "off_by_one", "no_saturation", "dropped_min"])
def test_planted_fw_mistakes_are_caught(kind):
    assert not _fw_pins_pass(lambda W: _fw_mutant(W, kind))


# ---------------------------------------------------------------------------
# last-hop predecessors (Sec. 2 pred[i][j]; Sec. 3.1 argmin)
# ---------------------------------------------------------------------------

def test_predecessors_vs_bruteforce(oracle):
    rng = np.random.default_rng(51)
    for trial in range(60):
        n = int(rng.integers(1, 8))
        W = rand_graph(rng, n, 0.5, 1, 6)            # small costs: many ties
        D = oracle.fw_i32(W)
        P = oracle.predecessors_i32(D, W, threads=1)
        hops = oracle.brute_last_hops(W.tolist())
        for i in range(n):
            for j in range(n):
                want = min(hops[i][j]) if hops[i][j] else -1
                assert P[i, j] == want, (trial, i, j, P[i, j], hops[i][j])


def test_predecessor_walks_have_the_shortest_length(oracle):
    rng = np.random.default_rng(52)
    n = 70
    W = rand_graph(rng, n, 0.05, 1, 100)
    D = oracle.fw_i32(W)
    P = oracle.predecessors_i32(D, W)
    for i in range(n):
        for j in range(n):
            w = oracle.walk_weight(W, P, i, j)
            if i != j and D[i, j] >= INF:
                assert w is None
            else:
                assert w == D[i, j]
    # a planted mistake (predecessors of the transposed problem) breaks a walk
    bad = oracle.predecessors_i32(D.T.copy(), W.T.copy())
    with pytest.raises(AssertionError):
        for i in range(n):
            for j in range(n):
                w = oracle.walk_weight(W, bad, i, j)
                assert w is None or w == D[i, j]


# ---------------------------------------------------------------------------
# property-based: Floyd-Warshall equals exhaustive enumeration
# ---------------------------------------------------------------------------

from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 6).flatmap(lambda n: st.lists(
    st.lists(st.one_of(st.just(INF), st.integers(0, 50), st.integers(400_000_000, INF - 1)), min_size=n, max_size=n),
    min_size=n, max_size=n)))
def test_fw_property_bruteforce(rows):
    import oracle
    W = np.array(rows, dtype=np.int32)
    np.fill_diagonal(W, 0)
    np.testing.assert_array_equal(oracle.fw_i32(W), np.array(oracle.brute_apsp(W.tolist()), dtype=np.int64))
