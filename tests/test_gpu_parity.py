"""GPU parity: every HIP entry point, called through the C ABI, against the
CPU oracle on the same seeded inputs.

int32 results must be bit-exact.  fp32 min-plus products are exact too (one
rounding per term, exact min), so they are compared bit for bit; fp32 APSP
results associate path sums differently from the oracle and are compared to
the fp64 oracle with |got - ref| <= 1e-5 * ref, with +inf and 0 exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30
RTOL = 1e-5


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_i32(rng, shape, inf_frac=0.3, hi=INF):
    v = rng.integers(0, hi + 1, size=shape, dtype=np.int64)
    v[rng.random(shape) < inf_frac] = INF
    return v.astype(np.int32)


def rand_f32(rng, shape, inf_frac=0.3):
    v = rng.uniform(0.0, 10.0, size=shape).astype(np.float32)
    v[rng.random(shape) < inf_frac] = np.inf
    return v


def rand_graph_i32(rng, n, p, lo=1, hi=1000):
    W = np.where(rng.random((n, n)) < p, rng.integers(lo, hi + 1, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


def rand_graph_f32(rng, n, p):
    W = np.where(rng.random((n, n)) < p, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


def assert_close_f32(got, ref64, rtol=RTOL):
    got = got.astype(np.float64)
    inf_g, inf_r = np.isinf(got), np.isinf(ref64)
    assert np.array_equal(inf_g, inf_r), "reachability differs"
    fin = ~inf_r
    err = np.abs(got[fin] - ref64[fin])
    assert (err <= rtol * ref64[fin]).all(), f"max rel err {np.max(err / np.maximum(ref64[fin], 1e-300))}"
    assert np.array_equal(got[fin] == 0, ref64[fin] == 0)


# ---------------------------------------------------------------------------
# min-plus product (Sec. 3, Eq. 2)
# ---------------------------------------------------------------------------

SHAPES = [(1, 1, 1), (5, 7, 3), (64, 64, 64), (128, 128, 128), (129, 130, 131),
          (200, 72, 333), (257, 255, 1000), (1000, 17, 8), (3, 1000, 700), (300, 300, 2)]


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("splitk", [True, False])
def test_minplus_i32_bitexact(native, dev, tile, splitk):
    rng = np.random.default_rng(100 + tile + splitk)
    for m, n, k in SHAPES:
        A, B, C = rand_i32(rng, (m, k)), rand_i32(rng, (k, n)), rand_i32(rng, (m, n), inf_frac=0.5)
        ref = oracle.minplus_i32(A, B, C)
        Cd = to_dev(C, dev)
        native.minplus_gemm(to_dev(A, dev), to_dev(B, dev), Cd, tile=tile, splitk=splitk)
        np.testing.assert_array_equal(host(Cd), ref, err_msg=f"{m}x{n}x{k} tile {tile}")


@pytest.mark.parametrize("tile", [64, 128])
def test_minplus_f32_bitexact(native, dev, tile):
    rng = np.random.default_rng(200 + tile)
    for m, n, k in SHAPES:
        A, B, C = rand_f32(rng, (m, k)), rand_f32(rng, (k, n)), rand_f32(rng, (m, n), inf_frac=0.5)
        ref = oracle.minplus_f32(A, B, C)
        Cd = to_dev(C, dev)
        native.minplus_gemm(to_dev(A, dev), to_dev(B, dev), Cd, tile=tile)
        np.testing.assert_array_equal(host(Cd), ref, err_msg=f"{m}x{n}x{k} tile {tile}")


def test_minplus_split_k_forced(native, dev):
    # few output tiles and a long reduction: the launcher splits K and merges
    # partial minima with atomic min; the result must not change
    rng = np.random.default_rng(300)
    for dt in ("i32", "f32"):
        A = rand_i32(rng, (70, 5000)) if dt == "i32" else rand_f32(rng, (70, 5000))
        B = rand_i32(rng, (5000, 90)) if dt == "i32" else rand_f32(rng, (5000, 90))
        C = rand_i32(rng, (70, 90), 1.0) if dt == "i32" else rand_f32(rng, (70, 90), 1.0)
        ref = oracle.minplus_i32(A, B, C) if dt == "i32" else oracle.minplus_f32(A, B, C)
        for splitk in (True, False):
            Cd = to_dev(C, dev)
            native.minplus_gemm(to_dev(A, dev), to_dev(B, dev), Cd, splitk=splitk)
            np.testing.assert_array_equal(host(Cd), ref)


def test_minplus_strided_and_unaligned(native, dev):
    rng = np.random.default_rng(301)
    m, n, k = 150, 190, 170
    for pad in (0, 3, 64):        # pad 3 makes every ld odd: unvectorised path
        A = rand_i32(rng, (m, k + pad))
        B = rand_i32(rng, (k, n + pad))
        C = rand_i32(rng, (m, n + pad), 0.6)
        ref = C.copy()
        ref[:, :n] = oracle.minplus_i32(A[:, :k], B[:, :n], C[:, :n])
        Ad, Bd, Cd = to_dev(A, dev), to_dev(B, dev), to_dev(C, dev)
        native.minplus_gemm(Ad[:, :k], Bd[:, :n], Cd[:, :n])
        np.testing.assert_array_equal(host(Cd), ref)


def test_minplus_degenerate(native, dev):
    rng = np.random.default_rng(302)
    C = rand_i32(rng, (6, 5))
    Cd = to_dev(C, dev)
    native.minplus_gemm(torch.zeros((6, 0), dtype=torch.int32, device=dev),
                        torch.zeros((0, 5), dtype=torch.int32, device=dev), Cd)
    np.testing.assert_array_equal(host(Cd), C)
    # tropical identity on the right: A (min,+) I = A
    I = np.full((40, 40), INF, np.int32)
    np.fill_diagonal(I, 0)
    A = rand_i32(rng, (33, 40))
    Cd = to_dev(np.full((33, 40), INF, np.int32), dev)
    native.minplus_gemm(to_dev(A, dev), to_dev(I, dev), Cd)
    np.testing.assert_array_equal(host(Cd), A)
    # saturation at the top of the range
    A = np.full((8, 8), INF, np.int32)
    B = np.full((8, 8), INF, np.int32)
    Cd = to_dev(np.full((8, 8), INF, np.int32), dev)
    native.minplus_gemm(to_dev(A, dev), to_dev(B, dev), Cd)
    assert (host(Cd) == INF).all()


# ---------------------------------------------------------------------------
# tile closure, blocked FW, R-Kleene, squaring
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("closure", ["kloop", "square"])
def test_closure_i32(native, dev, closure):
    rng = np.random.default_rng(400)
    for s in (1, 2, 3, 17, 31, 64, 65, 100, 127, 128):
        W = rand_graph_i32(rng, s, 0.08)
        D = to_dev(W, dev)
        native.apsp_closure(D, closure=closure)
        np.testing.assert_array_equal(host(D), oracle.fw_i32(W), err_msg=f"s={s}")


@pytest.mark.parametrize("closure", ["kloop", "square"])
def test_closure_f32(native, dev, closure):
    rng = np.random.default_rng(401)
    for s in (1, 5, 64, 99, 128):
        W = rand_graph_f32(rng, s, 0.1)
        D = to_dev(W, dev)
        native.apsp_closure(D, closure=closure)
        assert_close_f32(host(D), oracle.fw_f64(W.astype(np.float64)))


SIZES = [1, 2, 3, 31, 64, 65, 127, 128, 129, 200, 255, 256, 257, 1000]


@pytest.mark.parametrize("algo", ["fw", "rkleene", "square"])
@pytest.mark.parametrize("block", [64, 128])
def test_apsp_i32_bitexact(native, dev, algo, block):
    rng = np.random.default_rng(500 + block)
    fn = {"fw": native.apsp_fw, "rkleene": native.apsp_rkleene, "square": native.apsp_square}[algo]
    for n in SIZES:
        W = rand_graph_i32(rng, n, min(0.5, 4.0 / max(n, 1)))
        D = to_dev(W, dev)
        fn(D, block=block)
        np.testing.assert_array_equal(host(D), oracle.fw_i32(W, threads=8), err_msg=f"n={n}")


@pytest.mark.parametrize("algo", ["fw", "rkleene"])
def test_apsp_f32_tolerance(native, dev, algo):
    rng = np.random.default_rng(600)
    fn = native.apsp_fw if algo == "fw" else native.apsp_rkleene
    for n in (3, 65, 129, 257, 700):
        W = rand_graph_f32(rng, n, min(0.5, 4.0 / n))
        D = to_dev(W, dev)
        fn(D)
        assert_close_f32(host(D), oracle.fw_f64(W.astype(np.float64), threads=8))


def test_algorithms_agree_bitexact(native, dev):
    rng = np.random.default_rng(700)
    W = rand_graph_i32(rng, 777, 0.01)
    outs = []
    for fn, kw in ((native.apsp_fw, {}), (native.apsp_rkleene, {}), (native.apsp_square, {}),
                   (native.apsp_rkleene, {"cutover": 300}), (native.apsp_fw, {"closure": "square"}),
                   (native.apsp_solve, {})):
        D = to_dev(W, dev)
        fn(D, **kw)
        outs.append(host(D))
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_strided_matrix(native, dev):
    rng = np.random.default_rng(701)
    n = 300
    W = rand_graph_i32(rng, n, 0.02)
    big = np.full((n, n + 20), 7, np.int32)
    big[:, :n] = W
    Dd = to_dev(big, dev)
    native.apsp_rkleene(Dd[:, :n])
    out = host(Dd)
    np.testing.assert_array_equal(out[:, :n], oracle.fw_i32(W))
    assert (out[:, n:] == 7).all()


def test_saturation_and_unreachable(native, dev):
    # long chain whose total exceeds INF: distances beyond 2^30 saturate
    n = 300
    W = np.full((n, n), INF, np.int32)
    np.fill_diagonal(W, 0)
    for i in range(n - 1):
        W[i, i + 1] = 10_000_000
    for fn in (native.apsp_fw, native.apsp_rkleene):
        D = to_dev(W, dev)
        fn(D)
        np.testing.assert_array_equal(host(D), oracle.fw_i32(W))


def test_validate(native, dev):
    W = rand_graph_i32(np.random.default_rng(800), 50, 0.1)
    assert native.apsp_validate(to_dev(W, dev)) == 0
    bad = W.copy(); bad[3, 3] = 1
    assert native.apsp_validate(to_dev(bad, dev)) == 1
    bad = W.copy(); bad[1, 2] = -5
    assert native.apsp_validate(to_dev(bad, dev)) == 1
    bad = W.copy(); bad[1, 2] = INF + 1; bad[2, 1] = 2**31 - 1
    assert native.apsp_validate(to_dev(bad, dev)) == 2
    F = rand_graph_f32(np.random.default_rng(801), 50, 0.1)
    assert native.apsp_validate(to_dev(F, dev)) == 0
    bad = F.copy(); bad[0, 1] = np.nan; bad[1, 0] = -0.5; bad[2, 2] = np.inf
    assert native.apsp_validate(to_dev(bad, dev)) == 3


# ---------------------------------------------------------------------------
# the named workloads, in the configuration the benchmark times
# ---------------------------------------------------------------------------

def test_workload_n256_full(native, dev):
    wl = gg.SINGLE["n256_p0.1_i32"]
    W = wl.make()
    ref = oracle.fw_i32(W)
    for fn in (native.apsp_fw, native.apsp_rkleene, native.apsp_solve):
        D = to_dev(W, dev)
        fn(D)
        np.testing.assert_array_equal(host(D), ref)


def test_workload_n4096_sampled(native, dev):
    wl = gg.SINGLE["n4096_p0.05_i32"]
    W = wl.make()
    src = wl.sources()
    ref = oracle.dijkstra_i32(W, src)
    for fn in (native.apsp_fw, native.apsp_rkleene):
        D = to_dev(W, dev)
        fn(D)
        out = host(D)
        np.testing.assert_array_equal(out[src], ref)
        assert oracle.certificate_i32(W, out, rows=(0, 64)) == 0


@pytest.mark.parametrize("algo", ["rkleene", "fw"])
def test_workload_n16384_i32_sampled(native, dev, algo):
    wl = gg.SINGLE["n16384_p0.01_i32"]
    W = wl.make()
    src = wl.sources()
    ref = oracle.dijkstra_i32(W, src)
    D = to_dev(W, dev)
    (native.apsp_rkleene if algo == "rkleene" else native.apsp_fw)(D)
    out = host(D[torch.from_numpy(src).to(dev)])
    np.testing.assert_array_equal(out, ref)


def test_workload_n16384_f32_sampled(native, dev):
    wl = gg.SINGLE["n16384_p0.01_f32"]
    W = wl.make()
    src = wl.sources()
    ref = oracle.dijkstra_f64(W, src)
    D = to_dev(W, dev)
    native.apsp_rkleene(D)
    out = host(D[torch.from_numpy(src).to(dev)])
    assert_close_f32(out, ref)


@pytest.mark.parametrize("block", [64, 128])
def test_fw_schedules_agree(native, dev, block):
    """Blocked FW with the fused next-pivot step (default look-ahead), with
    squaring closures (look-ahead without the fused step) and without
    look-ahead: each bit-identical to the oracle, including ragged last bands
    and a leading dimension larger than n."""
    rng = np.random.default_rng(910 + block)
    for n in (3 * block + 1, 640, 1000, 1100):
        W = rand_graph_i32(rng, n, min(0.5, 5.0 / n))
        ref = oracle.fw_i32(W, threads=8)
        for kw in ({}, {"closure": "square"}, {"lookahead": False}):
            D = to_dev(W, dev)
            native.apsp_fw(D, block=block, **kw)
            np.testing.assert_array_equal(host(D), ref, err_msg=f"n={n} {kw}")
        big = np.full((n, n + 7), 5, np.int32)
        big[:, :n] = W
        Dd = to_dev(big, dev)
        native.apsp_fw(Dd[:, :n], block=block)
        out = host(Dd)
        np.testing.assert_array_equal(out[:, :n], ref, err_msg=f"strided n={n}")
        assert (out[:, n:] == 5).all()
    F = rand_graph_f32(rng, 900, 0.01)
    ref64 = oracle.fw_f64(F.astype(np.float64), threads=8)
    for kw in ({}, {"closure": "square"}):
        D = to_dev(F, dev)
        native.apsp_fw(D, block=block, **kw)
        assert_close_f32(host(D), ref64)
