"""The planner's device feature pass (edge count and weak connectivity by a
lock-free union-find) against host computations (numpy edge count, scipy
weak components), and apsp_solve's automatic plan: with the shipped cost
model loaded it runs exactly the candidate apsp_plan picks for those
features, and the result is exact."""
import math

import numpy as np
import pytest
import torch
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30


def host_features(W):
    n = W.shape[0]
    fin = (W < INF) if W.dtype == np.int32 else np.isfinite(W)
    m = int(fin.sum()) - n
    ii, jj = np.nonzero(fin)
    comps = connected_components(coo_matrix((np.ones(ii.size), (ii, jj)), shape=(n, n)), directed=True,
                                 connection="weak")[0] if n else 0
    dens = m / max(1, n * (n - 1))
    return [math.log2(max(n, 1)), math.log10(max(dens, 1e-9)), 0.0, 1.0 if comps <= 1 else 0.0]


def chain_graph(n, seed, extra=()):
    """A path through a random vertex order (weakly connected), plus extra edges."""
    rng = np.random.default_rng(seed)
    W = np.full((n, n), INF, np.int32)
    np.fill_diagonal(W, 0)
    perm = rng.permutation(n)
    W[perm[:-1], perm[1:]] = 5
    for a, b in extra:
        W[a, b] = 3
    return W


def cases():
    rng = np.random.default_rng(77)
    out = []
    for n, p in ((2, 0.0), (2, 1.0), (3, 0.3), (100, 0.0), (100, 0.01), (300, 0.005), (1000, 0.001), (1000, 0.2),
                 (4097, 0.0003)):
        W = np.where(rng.random((n, n)) < p, rng.integers(1, 100, (n, n)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
        out.append((f"rand{n}_{p}", W))
    out.append(("chain2000", chain_graph(2000, 1)))
    two = chain_graph(1500, 2)
    two[:, 700:] = INF        # cut: the first 700 vertices of the matrix lose every edge into the rest
    two[700:, :700] = INF
    np.fill_diagonal(two, 0)
    out.append(("two_parts", two))
    star = np.full((600, 600), INF, np.int32)
    np.fill_diagonal(star, 0)
    star[1:, 0] = 7           # every vertex points to 0
    out.append(("star_in", star))
    # three dense random blocks with no edge between them, in a shuffled vertex order
    blk = np.full((3001, 3001), INF, np.int32)
    for a, b in ((0, 1000), (1000, 2200), (2200, 3001)):
        blk[a:b, a:b] = np.where(rng.random((b - a, b - a)) < 0.05, rng.integers(1, 100, (b - a, b - a)), INF)
    perm = rng.permutation(3001)
    blk = blk[perm][:, perm]
    np.fill_diagonal(blk, 0)
    out.append(("three_blocks3001", np.ascontiguousarray(blk)))
    big = np.where(rng.random((4096, 4096)) < 0.05, rng.integers(1, 100, (4096, 4096)), INF).astype(np.int32)
    np.fill_diagonal(big, 0)
    out.append(("rand4096_0.05", big))
    F = np.where(rng.random((500, 500)) < 0.004, rng.uniform(0.1, 10, (500, 500)), np.inf).astype(np.float32)
    np.fill_diagonal(F, 0)
    out.append(("f32_500", F))
    # below 1024 vertices (one workgroup, forest in LDS): two dense halves
    # joined by one edge, then the same with the edge removed; n % 4 = 1
    # and fp32
    halves = np.full((701, 701), np.inf, np.float32)
    halves[:350, :350] = np.where(rng.random((350, 350)) < 0.05, 1.5, np.inf)
    halves[350:, 350:] = np.where(rng.random((351, 351)) < 0.05, 2.5, np.inf)
    np.fill_diagonal(halves, 0)
    bridged = halves.copy()
    bridged[700, 3] = 4.0
    out.append(("f32_halves701_bridged", bridged))
    out.append(("f32_halves701", halves))
    return out


@pytest.mark.parametrize("name,W", cases(), ids=[c[0] for c in cases()])
def test_features_match_host(native, dev, name, W):
    got = native.apsp_features(torch.from_numpy(W).to(dev))
    want = host_features(W)
    assert got[0] == pytest.approx(want[0], abs=1e-6)
    assert got[1] == pytest.approx(want[1], abs=1e-5)
    assert got[2] == 0.0
    assert got[3] == want[3], f"{name}: connected flag"


def test_features_strided_view(native, dev):
    """A matrix inside a wider buffer (row stride n + 3, rows not 16-byte
    aligned) gives the features of the matrix alone."""
    rng = np.random.default_rng(78)
    for n in (301, 999, 1027, 2050):
        W = np.where(rng.random((n, n)) < 0.003, rng.integers(1, 100, (n, n)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
        buf = torch.zeros((n, n + 3), dtype=torch.int32, device=dev)   # zeros outside: would count as edges
        buf[:, :n] = torch.from_numpy(W).to(dev)
        got = native.apsp_features(buf[:, :n])
        want = host_features(W)
        assert got[1] == pytest.approx(want[1], abs=1e-5)
        assert got[3] == want[3]


def test_features_one_vertex(native, dev):
    assert native.apsp_features(torch.zeros((1, 1), dtype=torch.int32, device=dev))[3] == 1.0


def test_auto_solve_runs_the_model_pick(native, dev):
    """The context loads the shipped model; apsp_solve() with no options runs
    the candidate apsp_plan picks for the device features, exactly."""
    import os
    assert os.path.exists(native.MODEL_PATH)
    native.apsp_costmodel_load(native.MODEL_PATH)     # earlier tests may have replaced it
    graphs = [g for g in gg.sweep() if g.n <= 2500][:8]
    picks = set()
    for sg in graphs:
        W = gg.sweep_graph_i32(sg)
        Wd = torch.from_numpy(W).to(dev)
        f = native.apsp_features(Wd)
        _, want = native.apsp_plan(sg.n, 10 ** f[1], 1, bool(f[3]))
        D = Wd.clone()
        native.apsp_solve(D)
        assert native.apsp_solve_choice() == want, f"g{sg.g}"
        picks.add(want)
        src = gg.dijkstra_sources(sg.n, sg.seed, 16)
        np.testing.assert_array_equal(D[torch.from_numpy(src).to(dev)].cpu().numpy(), oracle.dijkstra_i32(W, src))
    assert -1 not in picks
    # with any option set the size rule decides
    D = torch.from_numpy(gg.sweep_graph_i32(graphs[0])).to(dev)
    native.apsp_solve(D, lookahead=False)
    assert native.apsp_solve_choice() == -1


def test_auto_solve_f32_skips_packed(native, dev):
    native.apsp_costmodel_load(native.MODEL_PATH)
    rng = np.random.default_rng(78)
    n = 700
    F = np.where(rng.random((n, n)) < 0.01, rng.uniform(0.1, 10, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(F, 0)
    D = torch.from_numpy(F).to(dev)
    native.apsp_solve(D)
    c = native.apsp_solve_choice()
    assert c >= 0 and not (native.apsp_candidate(c).flags & native.FLAG_PACKED16)
    ref = oracle.fw_f64(F.astype(np.float64), threads=8)
    got = D.cpu().numpy().astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all()
