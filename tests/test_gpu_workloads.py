"""GPU parity on the sweep workload: every candidate plan of the library on
sweep graphs (chained and unchained, a range of n and p) against the oracle's
Dijkstra on sampled sources, bit for bit; plus randomised shapes for the
min-plus product (hypothesis)."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30


def sweep_selection(limit_n=3000, count=10):
    graphs = [g for g in gg.sweep() if g.n <= limit_n]
    chained = [g for g in graphs if g.chain][: count // 2]
    free = [g for g in graphs if not g.chain][: count // 2]
    return chained + free


@pytest.mark.parametrize("sg", sweep_selection(), ids=lambda g: f"g{g.g}_n{g.n}")
def test_sweep_graph_every_candidate(native, dev, sg):
    W = gg.sweep_graph_i32(sg)
    src = gg.dijkstra_sources(sg.n, sg.seed, 32)
    ref = oracle.dijkstra_i32(W, src)
    Wd = torch.from_numpy(W).to(dev)
    idx = torch.from_numpy(src).to(dev)
    for c in range(native.apsp_candidate_count()):
        D = Wd.clone()
        native.apsp_solve(D, opts=native.apsp_candidate(c))
        got = D[idx].cpu().numpy()
        np.testing.assert_array_equal(got, ref, err_msg=f"candidate {c}")


def test_planned_solve_matches(native, dev):
    # the shipped cost model picks a plan; whatever it picks must be exact
    import json, os
    from paper_2310_03983_amd import autotune
    model = json.load(open(os.path.join(os.path.dirname(autotune.__file__), "data", "costmodel_mlp.json")))
    autotune.install(model)
    for sg in sweep_selection(count=4):
        W = gg.sweep_graph_i32(sg)
        f = autotune.features(W)
        dens = 10 ** f[1]
        opts, choice = native.apsp_plan(sg.n, dens, 1, bool(f[3]))
        assert 0 <= choice < native.apsp_candidate_count()
        D = torch.from_numpy(W).to(dev)
        native.apsp_solve(D, opts=opts)
        src = gg.dijkstra_sources(sg.n, sg.seed, 16)
        np.testing.assert_array_equal(D[torch.from_numpy(src).to(dev)].cpu().numpy(), oracle.dijkstra_i32(W, src))


def test_f32_n4096(native, dev):
    W = gg.graph_f32(4096, 0.05, 0.1, 10.0, gg.graph_seed(2, 0))
    src = gg.dijkstra_sources(4096, 2, 32)
    ref = oracle.dijkstra_f64(W, src)
    for fn in (native.apsp_fw, native.apsp_rkleene, native.apsp_solve):
        D = torch.from_numpy(W).to(dev)
        fn(D)
        got = D[torch.from_numpy(src).to(dev)].cpu().numpy().astype(np.float64)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin)
        assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all()


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(m=st.integers(1, 300), n=st.integers(1, 300), k=st.integers(1, 300),
       inf_frac=st.sampled_from([0.0, 0.3, 0.9, 1.0]), pad=st.sampled_from([0, 1, 5]),
       tile=st.sampled_from(["auto", 64, 128]), seed=st.integers(0, 2**31 - 1))
def test_minplus_random_shapes(native, dev, m, n, k, inf_frac, pad, tile, seed):
    rng = np.random.default_rng(seed)
    def mat(r, c):
        v = rng.integers(0, INF + 1, (r, c + pad), dtype=np.int64)
        v[rng.random((r, c + pad)) < inf_frac] = INF
        return v.astype(np.int32)
    A, B, C = mat(m, k), mat(k, n), mat(m, n)
    ref = C.copy()
    ref[:, :n] = oracle.minplus_i32(A[:, :k], B[:, :n], C[:, :n])
    Ad, Bd, Cd = (torch.from_numpy(x).to(dev) for x in (A, B, C))
    native.minplus_gemm(Ad[:, :k], Bd[:, :n], Cd[:, :n], tile=tile)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Cd.cpu().numpy(), ref)
