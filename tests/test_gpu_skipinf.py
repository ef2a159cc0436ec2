"""GPU parity of APSP_FLAG_SKIP_INF (products skip reduction slices whose A
or B block is all INF): int32 bit-exact against the oracle, fp32 within
1e-5 of the fp64 oracle with and without skipping, on graphs
sparse enough that whole slices are INF, disconnected graphs and dense ones."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

INF = 1 << 30


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def graph(rng, n, p, hi=100, dtype=np.int32):
    mask = rng.random((n, n)) < p
    if dtype == np.int32:
        W = np.where(mask, rng.integers(1, hi + 1, (n, n)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
    else:
        W = np.where(mask, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
        np.fill_diagonal(W, 0.0)
    return W


CASES = [(1, 0.5), (2, 0.0), (100, 0.0), (129, 0.002), (300, 0.0005), (700, 0.001), (1000, 0.003),
         (257, 0.05), (512, 0.5)]


@pytest.mark.parametrize("algo", ["fw", "rkleene", "square"])
def test_skip_inf_i32_bitexact(native, dev, algo):
    rng = np.random.default_rng(2000)
    fn = {"fw": native.apsp_fw, "rkleene": native.apsp_rkleene, "square": native.apsp_square}[algo]
    for n, p in CASES:
        W = graph(rng, n, p)
        ref = oracle.fw_i32(W, threads=8)
        for kw in ({"skip_inf": True}, {"skip_inf": True, "block": 64}, {"skip_inf": True, "packed16": True},
                   {"skip_inf": True, "cutover": 256}, {"skip_inf": True, "tile": 128}):
            D = to_dev(W, dev)
            fn(D, **kw)
            np.testing.assert_array_equal(host(D), ref, err_msg=f"n={n} p={p} {kw}")


def test_skip_inf_f32_oracle(native, dev):
    """fp32 with and without skipping, each against the fp64 oracle (1e-5
    relative; +inf and 0 exact).  In-place fp32 R-Kleene may round path sums
    differently from run to run, so the two runs are not compared bit for bit."""
    rng = np.random.default_rng(2001)
    for n, p in ((300, 0.001), (700, 0.002), (513, 0.05)):
        W = graph(rng, n, p, dtype=np.float32)
        ref = oracle.fw_f64(W.astype(np.float64), threads=8)
        fin = np.isfinite(ref)
        for algo in ("fw", "rkleene"):
            for skip in (False, True):
                D = to_dev(W, dev)
                (native.apsp_fw if algo == "fw" else native.apsp_rkleene)(D, skip_inf=skip)
                got = host(D).astype(np.float64)
                what = f"n={n} {algo} skip={skip}"
                assert np.array_equal(np.isfinite(got), fin), what
                assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all(), what
                assert np.array_equal(got[fin] == 0, ref[fin] == 0), what


def test_skip_inf_minplus_gemm(native, dev):
    rng = np.random.default_rng(2002)
    for m, n, k, pa, pb in ((300, 200, 500, 0.001, 0.5), (256, 256, 256, 0.0, 0.3), (129, 513, 70, 0.02, 0.02)):
        A = graph(rng, max(m, k), pa)[:m, :k].copy()
        B = graph(rng, max(k, n), pb)[:k, :n].copy()
        C = graph(rng, max(m, n), 0.01)[:m, :n].copy()
        ref = oracle.minplus_i32(A, B, C)
        Cd = to_dev(C, dev)
        native.minplus_gemm(to_dev(A, dev), to_dev(B, dev), Cd, skip_inf=True)
        np.testing.assert_array_equal(host(Cd), ref, err_msg=f"{m}x{n}x{k}")
