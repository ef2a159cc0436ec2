"""GPU parity of the predecessor kernel (Sec. 2 pred, Sec. 3.1 argmin)
against the oracle: bit-exact for int32, validity for fp32, and paths rebuilt
from P have the shortest length."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30


def rand_graph(rng, n, p, lo=1, hi=100):
    W = np.where(rng.random((n, n)) < p, rng.integers(lo, hi + 1, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


def test_predecessors_i32_bitexact(native, dev):
    rng = np.random.default_rng(1000)
    for n in (1, 2, 3, 31, 63, 64, 65, 200, 301):
        W = rand_graph(rng, n, min(0.5, 3.0 / n), 1, 8)      # small costs: many ties
        D = oracle.fw_i32(W)
        Pd = native.apsp_predecessors(torch.from_numpy(D).to(dev), torch.from_numpy(W).to(dev))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Pd.cpu().numpy(), oracle.predecessors_i32(D, W), err_msg=f"n={n}")


def test_paths_from_gpu_solve(native, dev):
    wl = gg.SINGLE["n256_p0.1_i32"]
    W = wl.make()
    Wd = torch.from_numpy(W).to(dev)
    D = Wd.clone()
    native.apsp_solve(D)
    P = native.apsp_predecessors(D, Wd)
    torch.cuda.synchronize()
    Dh, Ph = D.cpu().numpy(), P.cpu().numpy()
    np.testing.assert_array_equal(Ph, oracle.predecessors_i32(oracle.fw_i32(W), W))
    for i in range(0, 256, 17):
        paths = native.apsp_path(P, [i] * 256, list(range(256)))
        for j, path in enumerate(paths):
            if Dh[i, j] >= INF:
                assert path == []
            else:
                assert path[0] == i and path[-1] == j
                assert sum(int(W[a, b]) for a, b in zip(path, path[1:])) == Dh[i, j]


def test_predecessors_n4096_sampled_rows(native, dev):
    wl = gg.SINGLE["n4096_p0.05_i32"]
    W = wl.make()
    Wd = torch.from_numpy(W).to(dev)
    D = Wd.clone()
    native.apsp_solve(D)
    P = native.apsp_predecessors(D, Wd)
    torch.cuda.synchronize()
    rows = wl.sources(8)
    Dh = D.cpu().numpy().astype(np.int64)
    Ph = P.cpu().numpy()
    Wm = W.astype(np.int64).copy()
    np.fill_diagonal(Wm, INF)                       # v == j is excluded
    for i in rows:
        # definition, vectorised over j: smallest v minimising D[i][v] (+) W[v][j]
        cand = np.minimum(Dh[i][:, None] + Wm, INF)
        want = np.argmin(cand, axis=0).astype(np.int32)
        want[cand.min(axis=0) >= INF] = -1
        want[i] = -1
        np.testing.assert_array_equal(Ph[i], want)


def test_predecessors_f32_valid(native, dev):
    rng = np.random.default_rng(1001)
    n = 300
    W = np.where(rng.random((n, n)) < 0.02, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    Wd = torch.from_numpy(W).to(dev)
    D = Wd.clone()
    native.apsp_solve(D)
    P = native.apsp_predecessors(D, Wd)
    torch.cuda.synchronize()
    Dh, Ph = D.cpu().numpy().astype(np.float64), P.cpu().numpy()
    ref = oracle.fw_f64(W.astype(np.float64))
    for i in range(n):
        paths = native.apsp_path(P, [i] * n, list(range(n)))
        for j in range(n):
            if i == j or np.isinf(ref[i, j]):
                assert Ph[i, j] == -1
                continue
            path = paths[j]
            w = sum(float(W[a, b]) for a, b in zip(path, path[1:]))
            assert abs(w - ref[i, j]) <= 1e-5 * ref[i, j]


def run_form(native, D, W, dev, method):
    P = native.apsp_predecessors(torch.from_numpy(D).to(dev), torch.from_numpy(W).to(dev), method=method)
    torch.cuda.synchronize()
    return P.cpu().numpy()


@pytest.mark.parametrize("closure", [True, False])
def test_predecessor_forms_agree_i32(native, dev, closure):
    """Dense, sparse and automatic forms give the oracle's P, for D the
    closure of W and for an arbitrary D (the definition covers any D)."""
    rng = np.random.default_rng(1100 + closure)
    for n, p in ((1, 0.5), (2, 1.0), (3, 0.0), (63, 0.05), (64, 0.3), (65, 1.0), (300, 0.01),
                 (1023, 0.004), (1024, 0.02), (1025, 0.002), (1100, 0.0)):
        W = rand_graph(rng, n, p, 1, 8)                         # small costs: many ties
        if closure:
            D = oracle.fw_i32(W)
        else:
            D = rng.integers(0, 40, (n, n)).astype(np.int32)
            D[rng.random((n, n)) < 0.2] = INF
        ref = oracle.predecessors_i32(D, W)
        for method in ("dense", "sparse", "auto"):
            np.testing.assert_array_equal(run_form(native, D, W, dev, method), ref, err_msg=f"n={n} p={p} {method}")


def test_predecessor_forms_agree_f32(native, dev):
    rng = np.random.default_rng(1200)
    for n, p in ((5, 0.5), (130, 0.05), (1030, 0.01)):
        W = np.where(rng.random((n, n)) < p, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
        np.fill_diagonal(W, 0.0)
        Wd = torch.from_numpy(W).to(dev)
        D = Wd.clone()
        native.apsp_solve(D)
        Dh = D.cpu().numpy()
        dense = run_form(native, Dh, W, dev, "dense")
        np.testing.assert_array_equal(run_form(native, Dh, W, dev, "sparse"), dense, err_msg=f"n={n}")


def test_predecessor_forms_agree_n4096(native, dev):
    wl = gg.SINGLE["n4096_p0.05_i32"]
    W = wl.make()
    Wd = torch.from_numpy(W).to(dev)
    D = Wd.clone()
    native.apsp_solve(D)
    Ps = native.apsp_predecessors(D, Wd, method="sparse")
    Pd = native.apsp_predecessors(D, Wd, method="dense")
    torch.cuda.synchronize()
    assert torch.equal(Ps, Pd)


def test_path_walks(native, dev):
    """apsp_path on a hand-made predecessor matrix: rows 0 and 1 encode
    0->1->2, 0->1->3 with 4 unreachable from 0; row 2 has a cycle 0 <- 1 <- 0
    that never reaches 2 (a broken chain)."""
    P = np.full((5, 5), -1, np.int32)
    P[0] = [-1, 0, 1, 1, -1]
    P[2] = [1, 0, -1, 2, 2]
    Pd = torch.from_numpy(P).to(dev)
    assert native.apsp_path(Pd, 0, 2) == [0, 1, 2]
    assert native.apsp_path(Pd, 0, 3) == [0, 1, 3]
    assert native.apsp_path(Pd, 0, 4) == []
    assert native.apsp_path(Pd, 0, 0) == [0]
    assert native.apsp_path(Pd, [0, 0, 0], [1, 3, 0]) == [[0, 1], [0, 1, 3], [0]]
    with pytest.raises(ValueError):
        native.apsp_path(Pd, 2, 0)          # 0 <- 1 <- 0 ... never reaches 2
    with pytest.raises(ValueError):
        native.apsp_path(Pd, 0, 3, max_len=2)   # the path has 3 vertices
    with pytest.raises(ValueError):
        native.apsp_path(Pd, 0, 7)          # target out of range
    assert native.apsp_path(Pd, [], []) == []


def test_sparse_form_workspace(native, dev):
    """The sparse form lives in the caller's workspace: without one, AUTO runs
    the dense form and SPARSE is APSP_E_NOMEM; with a workspace too small for
    the edge list the device falls back to the dense form; the results never
    change."""
    import ctypes
    rng = np.random.default_rng(1300)
    n = 700
    W = rand_graph(rng, n, 0.02, 1, 8)
    D = oracle.fw_i32(W)
    ref = oracle.predecessors_i32(D, W)
    Dd, Wd = torch.from_numpy(D).to(dev), torch.from_numpy(W).to(dev)
    L = native.lib()
    ctx = native.context(dev.index)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(method):
        P = torch.full((n, n), 7, dtype=torch.int32, device=dev)
        rc = L.apsp_predecessors_ex(ctx, 0, n, Dd.data_ptr(), n, Wd.data_ptr(), n, P.data_ptr(), n,
                                    native.PRED[method], st)
        torch.cuda.synchronize()
        return rc, P.cpu().numpy()

    saved = native._ws.get(dev.index)
    try:
        native.apsp_set_workspace(None, dev.index)
        rc, P = call("auto")
        assert rc == native.APSP_OK
        np.testing.assert_array_equal(P, ref)
        rc, _ = call("sparse")
        assert rc == native.APSP_E_NOMEM and "workspace" in native.last_error()
        full = native.apsp_workspace_size("predecessors", n)
        m = int((W < INF).sum()) - n
        # 16 KB: above the fixed part at n = 700 (flag 256 B, counts 3 KB,
        # offsets 5.5 KB) but room for only ~900 of the ~9800 edges, so the
        # device falls back to the dense form
        small = torch.empty(16384, dtype=torch.uint8, device=dev)
        native.apsp_set_workspace(small, dev.index)
        for method in ("auto", "sparse"):
            rc, P = call(method)
            assert rc == native.APSP_OK
            np.testing.assert_array_equal(P, ref, err_msg=method)
        big = torch.empty(full, dtype=torch.uint8, device=dev)
        native.apsp_set_workspace(big, dev.index)
        for method in ("auto", "sparse", "dense"):
            rc, P = call(method)
            assert rc == native.APSP_OK
            np.testing.assert_array_equal(P, ref, err_msg=method)
        assert m > 2000
    finally:
        native.apsp_set_workspace(saved, dev.index)
