"""APSP_FLAG_DETERMINISTIC (reading 9 of the design: in-place fp32 products
may round path sums differently from run to run): with the flag, every
product whose output block is also an operand reads a copy taken first, so
fp32 results are identical bit for bit from run to run -- checked over
repeated runs of R-Kleene (recursion to the leaves and with an FW cutover)
and blocked FW at sizes with many such products, each run also within
1e-5 of the fp64 oracle; int32 results stay equal to the oracle's."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

INF = 1 << 30


def threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(os.cpu_count() or 1, 16)


def f32_graph(rng, n, p):
    W = np.where(rng.random((n, n)) < p, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


def close_f32(got, ref):
    got = got.astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all()


CASES = [("rkleene", 2500, 0.01, {"cutover": 0}), ("rkleene", 3000, 0.005, {"cutover": 1024}),
         ("fw", 1500, 0.01, {}), ("fw", 1100, 0.02, {"block": 64})]


@pytest.mark.parametrize("algo,n,p,kw", CASES, ids=[f"{a}{n}_{i}" for i, (a, n, p, kw) in enumerate(CASES)])
def test_f32_bit_identical_runs(native, dev, algo, n, p, kw):
    rng = np.random.default_rng(n + 31)
    W = f32_graph(rng, n, p)
    ref = oracle.fw_f64(W.astype(np.float64), threads=threads())
    fn = native.apsp_rkleene if algo == "rkleene" else native.apsp_fw
    Wd = torch.from_numpy(W).to(dev)
    runs = []
    for _ in range(4):
        D = Wd.clone()
        fn(D, deterministic=True, **kw)
        torch.cuda.synchronize()
        runs.append(D.cpu().numpy())
    for r in runs[1:]:
        assert np.array_equal(r.view(np.uint32), runs[0].view(np.uint32)), f"{algo} n={n} {kw}"
    close_f32(runs[0], ref)


def test_i32_deterministic_equals_oracle(native, dev):
    rng = np.random.default_rng(77)
    n = 1300
    W = np.where(rng.random((n, n)) < 0.01, rng.integers(1, 1000, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    ref = oracle.fw_i32(W, threads=threads())
    for fn, kw in ((native.apsp_rkleene, {"cutover": 0}), (native.apsp_fw, {}), (native.apsp_solve, {})):
        D = torch.from_numpy(W).to(dev)
        fn(D, deterministic=True, **kw)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(D.cpu().numpy(), ref)


def test_square_rejects_the_flag(native, dev):
    D = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    with pytest.raises(native.ApspError) as e:
        native.apsp_square(D, deterministic=True)
    assert e.value.status == native.APSP_E_UNSUPPORTED
