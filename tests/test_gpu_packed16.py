"""GPU parity of the capped 16-bit mode (APSP_FLAG_PACKED16) through the C ABI.

The mode must return exactly the int32 result in every case: compared bit for
bit with the CPU oracle, both when every distance stays below the cap (no
int32 redo) and when some entry reaches it (unreachable pairs, long paths,
edge costs above the cap, saturation at INF), which forces the int32 redo.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30
CAP = 0x39FF   # the cap of the packed products (apsp.CAP16)
FNS = ("fw", "rkleene", "square")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver(native, algo):
    return {"fw": native.apsp_fw, "rkleene": native.apsp_rkleene, "square": native.apsp_square,
            "solve": native.apsp_solve}[algo]


def cycle_graph(rng, n, p, hi):
    """Random graph plus the cycle 0 -> 1 -> ... -> n-1 -> 0, so every vertex
    reaches every other; costs in [1, hi]."""
    W = np.where(rng.random((n, n)) < p, rng.integers(1, hi + 1, (n, n)), INF).astype(np.int32)
    idx = np.arange(n)
    W[idx, (idx + 1) % n] = rng.integers(1, hi + 1, n)
    np.fill_diagonal(W, 0)
    return W


def run(native, algo, W, dev, **kw):
    D = to_dev(W, dev)
    before = native.apsp_packed16_counts()
    solver(native, algo)(D, packed16=True, **kw)
    after = native.apsp_packed16_counts()
    return host(D), after[0] - before[0], after[1] - before[1]


SIZES = [2, 3, 31, 64, 65, 127, 128, 129, 200, 257, 1000]


@pytest.mark.parametrize("algo", FNS)
@pytest.mark.parametrize("block", [64, 128])
def test_packed16_exact_without_redo(native, dev, algo, block):
    rng = np.random.default_rng(1600 + block)
    for n in SIZES:
        W = cycle_graph(rng, n, min(0.5, 4.0 / n), 20)   # distances <= 20 (n - 1) < CAP
        ref = oracle.fw_i32(W, threads=8)
        assert ref.max() < CAP
        out, runs, redone = run(native, algo, W, dev, block=block)
        np.testing.assert_array_equal(out, ref, err_msg=f"n={n}")
        assert (runs, redone) == (1, 0), f"n={n}"


@pytest.mark.parametrize("algo", FNS)
def test_packed16_redo_cases(native, dev, algo):
    rng = np.random.default_rng(1700)
    cases = []
    # unreachable pairs
    W = np.where(rng.random((300, 300)) < 0.004, rng.integers(1, 100, (300, 300)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    cases.append(("disconnected", W))
    # every vertex reachable, but long paths pass the cap
    cases.append(("long paths", cycle_graph(rng, 257, 0.002, 3000)))
    # edge costs above the cap mixed with small ones
    W = cycle_graph(rng, 200, 0.05, 50)
    heavy = rng.random(W.shape) < 0.05
    W[heavy] = rng.integers(CAP, 200_000, int(heavy.sum()))
    np.fill_diagonal(W, 0)
    cases.append(("heavy edges", W))
    # a chain whose sums saturate at INF
    W = np.full((300, 300), INF, np.int32)
    np.fill_diagonal(W, 0)
    W[np.arange(299), np.arange(1, 300)] = 10_000_000
    cases.append(("saturating chain", W))
    for name, W in cases:
        ref = oracle.fw_i32(W, threads=8)
        out, runs, redone = run(native, algo, W, dev)
        np.testing.assert_array_equal(out, ref, err_msg=name)
        assert runs == 1
        assert redone == (1 if (ref >= CAP).any() else 0), name


def test_packed16_tiles_and_split(native, dev):
    rng = np.random.default_rng(1800)
    W = cycle_graph(rng, 1000, 0.01, 30)
    ref = oracle.fw_i32(W, threads=8)
    for kw in ({"tile": 64}, {"tile": 128}, {"tile": 128, "splitk": False},
               {"cutover": 300}, {"closure": "square"}, {"lookahead": False}):
        for algo in ("fw", "rkleene"):
            out, _, redone = run(native, algo, W, dev, **kw)
            np.testing.assert_array_equal(out, ref, err_msg=f"{algo} {kw}")
            assert redone == 0


def test_packed16_strided(native, dev):
    rng = np.random.default_rng(1801)
    n = 300
    W = cycle_graph(rng, n, 0.02, 40)
    big = np.full((n, n + 13), 7, np.int32)
    big[:, :n] = W
    Dd = to_dev(big, dev)
    native.apsp_rkleene(Dd[:, :n], packed16=True)
    out = host(Dd)
    np.testing.assert_array_equal(out[:, :n], oracle.fw_i32(W))
    assert (out[:, n:] == 7).all()


def test_packed16_agrees_with_int32_n4096(native, dev):
    wl = gg.SINGLE["n4096_p0.05_i32"]
    W = wl.make()
    outs = []
    for flag in (False, True):
        D = to_dev(W, dev)
        native.apsp_solve(D, packed16=flag)
        outs.append(host(D))
    np.testing.assert_array_equal(outs[1], outs[0])
    src = wl.sources()
    np.testing.assert_array_equal(outs[1][src], oracle.dijkstra_i32(W, src))


def test_packed16_workload_n16384_sampled(native, dev):
    wl = gg.SINGLE["n16384_p0.01_i32"]
    W = wl.make()
    src = wl.sources()
    ref = oracle.dijkstra_i32(W, src)
    D = to_dev(W, dev)
    before = native.apsp_packed16_counts()
    native.apsp_rkleene(D, cutover=4096, packed16=True)
    after = native.apsp_packed16_counts()
    out = host(D[torch.from_numpy(src).to(dev)])
    np.testing.assert_array_equal(out, ref)
    assert after[1] == before[1], "every distance of this workload is below the cap"


def test_cap_constant_matches_binding(native):
    assert native.CAP16 == CAP


def test_packed16_rejected_for_f32(native, dev):
    F = np.zeros((8, 8), np.float32)
    with pytest.raises(native.ApspError) as e:
        native.apsp_fw(to_dev(F, dev), packed16=True)
    assert e.value.status == native.APSP_E_UNSUPPORTED


@pytest.mark.parametrize("algo", FNS)
def test_packed16_random_graphs(native, dev, algo):
    """Random graphs across the cap: every result bit-identical to the oracle,
    and the int32 redo runs exactly when some true distance reaches the cap."""
    from hypothesis import given, settings, HealthCheck, strategies as st

    @settings(max_examples=12, deadline=None, suppress_health_check=list(HealthCheck), derandomize=True)
    @given(n=st.integers(2, 300), logp=st.floats(-3.0, 0.0), hi=st.sampled_from([5, 200, 3000, 60000]),
           seed=st.integers(0, 2**31))
    def check(n, logp, hi, seed):
        rng = np.random.default_rng(seed)
        p = 10.0 ** logp
        W = np.where(rng.random((n, n)) < p, rng.integers(1, hi + 1, (n, n)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
        ref = oracle.fw_i32(W, threads=8)
        out, runs, redone = run(native, algo, W, dev)
        np.testing.assert_array_equal(out, ref, err_msg=f"n={n} p={p:.3g} hi={hi}")
        assert runs == 1 and redone == int((ref >= CAP).any())

    check()
