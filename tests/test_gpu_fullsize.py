"""Whole-matrix parity at the full workload sizes.

Every entry of every large result is checked, not a sample of rows:

* n = 16384, int32 (costs 1..1000, p = 0.01): the R-Kleene result is
  certified entry by entry with the oracle's Bellman certificate (conditions
  on every edge and every target; exactly the closure iff all hold, since
  every cost is >= 1), and the blocked-FW, capped-16-bit and default-solve
  results must equal it bit for bit;
* n = 16384, fp32 (costs 0.1..10.0): every row against fp64 Dijkstra from
  that source, |got - ref| <= 1e-5 ref, +inf and 0 exact;
* n = 4096, int32: the full triple-loop oracle (Sec. 2, Eq. 1) and the
  certificate over all rows, for every solver;
* two sweep graphs above n = 8192, every candidate plan, against Dijkstra.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(os.cpu_count() or 1, 16)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_close_f32(got, ref64, what):
    got = got.astype(np.float64)
    inf_g, inf_r = np.isinf(got), np.isinf(ref64)
    assert np.array_equal(inf_g, inf_r), f"{what}: reachability differs"
    fin = ~inf_r
    err = np.abs(got[fin] - ref64[fin])
    assert (err <= RTOL * ref64[fin]).all(), f"{what}: max rel err {np.max(err / np.maximum(ref64[fin], 1e-300))}"
    assert np.array_equal(got[fin] == 0, ref64[fin] == 0), f"{what}: zero pattern differs"


def test_n16384_i32_whole_matrix(native, dev):
    wl = gg.SINGLE["n16384_p0.01_i32"]
    W = wl.make()
    print(f"n16384 int32: certificate over all rows, {threads()} threads", flush=True)
    Wd = torch.from_numpy(W).to(dev)
    D = Wd.clone()
    native.apsp_rkleene(D, cutover=4096)
    ref = host(D)
    assert oracle.certificate_i32(W, ref, threads=threads()) == 0
    del D
    cases = (("fw", native.apsp_fw, {}),
             ("rkleene packed16", native.apsp_rkleene, {"cutover": 4096, "packed16": True}),
             ("fw packed16", native.apsp_fw, {"packed16": True}),
             ("solve default", native.apsp_solve, {}))
    for name, fn, kw in cases:
        D = Wd.clone()
        fn(D, **kw)
        got = host(D)
        del D
        bad = int((got != ref).sum())
        assert bad == 0, f"{name}: {bad} entries differ from the certified matrix"


def test_n16384_f32_every_row(native, dev):
    wl = gg.SINGLE["n16384_p0.01_f32"]
    W = wl.make()
    n = W.shape[0]
    D = torch.from_numpy(W).to(dev)
    native.apsp_rkleene(D)
    got = host(D)
    del D
    chunk = 2048
    print(f"n16384 fp32: fp64 Dijkstra from all {n} sources, {threads()} threads", flush=True)
    for s0 in range(0, n, chunk):
        src = np.arange(s0, min(n, s0 + chunk), dtype=np.int64)
        ref = oracle.dijkstra_f64(W, src, threads=threads())
        assert_close_f32(got[src], ref, f"rows {s0}..{src[-1]}")


def test_n4096_i32_full_oracle(native, dev):
    wl = gg.SINGLE["n4096_p0.05_i32"]
    W = wl.make()
    print(f"n4096 int32: full triple-loop oracle, {threads()} threads", flush=True)
    ref = oracle.fw_i32(W, threads=threads())
    assert oracle.certificate_i32(W, ref, threads=threads()) == 0
    Wd = torch.from_numpy(W).to(dev)
    cases = (("fw", native.apsp_fw, {}), ("fw b64", native.apsp_fw, {"block": 64}),
             ("rkleene", native.apsp_rkleene, {}), ("solve", native.apsp_solve, {}),
             ("fw packed16", native.apsp_fw, {"packed16": True}),
             ("square", native.apsp_square, {}))
    for name, fn, kw in cases:
        D = Wd.clone()
        fn(D, **kw)
        got = host(D)
        bad = int((got != ref).sum())
        assert bad == 0, f"{name}: {bad} entries differ from the oracle"
        assert oracle.certificate_i32(W, got, threads=threads()) == 0, name


BIG_SWEEP = (2, 29)   # n = 14821 (chained, p = 0.0018), n = 13664 (unchained, p = 0.00276)


@pytest.mark.parametrize("g", BIG_SWEEP)
def test_big_sweep_graph_every_candidate(native, dev, g):
    sg = gg.sweep()[g]
    assert sg.n > 8192
    W = gg.sweep_graph_i32(sg)
    src = gg.dijkstra_sources(sg.n, sg.seed, 32)
    ref = oracle.dijkstra_i32(W, src, threads=threads())
    Wd = torch.from_numpy(W).to(dev)
    idx = torch.from_numpy(src).to(dev)
    first = None
    for c in range(native.apsp_candidate_count()):
        print(f"sweep g{g} n={sg.n}: candidate {c}", flush=True)
        D = Wd.clone()
        native.apsp_solve(D, opts=native.apsp_candidate(c))
        np.testing.assert_array_equal(host(D[idx]), ref, err_msg=f"candidate {c}")
        # every candidate's whole matrix equals candidate 0's
        if first is None:
            first = D
        else:
            assert torch.equal(D, first), f"candidate {c} differs from candidate 0"
        del D
