"""GPU parity of whole-graph squaring (Sec. 3.2) in its one-launch form
(apsp_square for n <= 2048: every pass inside one launch, tasks of a pass
waiting on the previous pass's counter, convergence detected on the
device): int32 bit-exact against the oracle's Eq. 1 loop, fp32 within 1e-5
of the fp64 oracle, on graphs that need the most passes (a path through
every vertex), disconnected graphs, strided views, ragged sizes on both
tile sizes, and back-to-back calls (the counters are reset per launch);
the reported pass count stays within ceil(log2(n - 1))."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

INF = 1 << 30


def threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(os.cpu_count() or 1, 16)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_i32(rng, n, p, hi=100):
    W = np.where(rng.random((n, n)) < p, rng.integers(1, hi + 1, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


def path_i32(rng, n):
    """A path through every vertex in a random order plus a few far-apart
    shortcuts of high cost: the longest shortest path has n - 1 edges, so
    the pass bound is reached."""
    W = np.full((n, n), INF, np.int32)
    np.fill_diagonal(W, 0)
    perm = rng.permutation(n)
    W[perm[:-1], perm[1:]] = rng.integers(1, 10, n - 1)
    a, b = rng.integers(0, n, 8), rng.integers(0, n, 8)
    W[a, b] = np.where(a != b, 50 * n, 0)
    return W


CASES = [("rand", 3, 0.5), ("rand", 4, 0.0), ("rand", 63, 0.2), ("rand", 64, 0.05), ("rand", 65, 0.05),
         ("rand", 200, 0.02), ("rand", 256, 0.1), ("rand", 257, 0.003), ("path", 300, 0), ("rand", 400, 0.02), ("path", 450, 0), ("rand", 511, 0.02),
         ("rand", 512, 0.3), ("path", 512, 0), ("rand", 700, 0.01),
         ("path", 1024, 0), ("rand", 1024, 0.002), ("rand", 1500, 0.004), ("rand", 2048, 0.01), ("path", 2048, 0)]


@pytest.mark.parametrize("kind,n,p", CASES, ids=[f"{k}{n}_{p}" for k, n, p in CASES])
def test_square_i32_bitexact(native, dev, kind, n, p):
    rng = np.random.default_rng(n * 7 + int(p * 1e4))
    W = rand_i32(rng, n, p) if kind == "rand" else path_i32(rng, n)
    ref = oracle.fw_i32(W, threads=threads())
    D = torch.from_numpy(W).to(dev)
    native.apsp_square(D)
    np.testing.assert_array_equal(host(D), ref, err_msg=f"{kind} n={n} p={p}")
    bound = int(np.ceil(np.log2(n - 1))) if n > 2 else 0
    passes = native.apsp_square_passes()
    assert (1 if n > 2 else 0) <= passes <= bound, (passes, bound)


def test_square_strided_and_back_to_back(native, dev):
    """Two calls in a row on views with row stride n + 5 inside a buffer
    whose other columns must stay untouched; then a smaller graph."""
    rng = np.random.default_rng(4242)
    for n in (513, 129):
        W = rand_i32(rng, n, 0.01)
        ref = oracle.fw_i32(W, threads=threads())
        buf = torch.full((n, n + 5), 77, dtype=torch.int32, device=dev)
        buf[:, :n] = torch.from_numpy(W).to(dev)
        native.apsp_square(buf[:, :n])
        out = host(buf)
        np.testing.assert_array_equal(out[:, :n], ref, err_msg=f"n={n}")
        assert (out[:, n:] == 77).all()


def test_square_disconnected(native, dev):
    rng = np.random.default_rng(4243)
    n = 600
    W = rand_i32(rng, n, 0.02)
    W[:300, 300:] = INF   # no edge from the first half into the second
    ref = oracle.fw_i32(W, threads=threads())
    D = torch.from_numpy(W).to(dev)
    native.apsp_square(D)
    got = host(D)
    np.testing.assert_array_equal(got, ref)
    assert (got[:300, 300:] == INF).all()


@pytest.mark.parametrize("n,p", [(5, 0.5), (256, 0.1), (512, 0.02), (777, 0.01), (2048, 0.005)])
def test_square_f32_oracle(native, dev, n, p):
    rng = np.random.default_rng(4244 + n)
    W = np.where(rng.random((n, n)) < p, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    ref = oracle.fw_f64(W.astype(np.float64), threads=threads())
    D = torch.from_numpy(W).to(dev)
    native.apsp_square(D)
    got = host(D).astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all()
    assert np.array_equal(got[fin] == 0, ref[fin] == 0)
