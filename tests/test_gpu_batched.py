"""GPU parity of the batched path: every graph of a ragged batch, solved in
one persistent launch (replayed from a captured HIP graph), against the CPU
oracle, bit for bit for int32."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_03983_amd import graphgen as gg

pytestmark = pytest.mark.gpu

INF = 1 << 30


def pack(mats, dev):
    flat, off, sz = gg.pack_batch(mats)
    return (torch.from_numpy(flat).to(dev), torch.from_numpy(off).to(dev),
            torch.from_numpy(sz).to(dev), sz.tolist(), off)


def unpack(flat_d, off, sizes):
    torch.cuda.synchronize()
    flat = flat_d.cpu().numpy()
    return [flat[o:o + n * n].reshape(n, n) for o, n in zip(off, sizes)]


def rand_graph(rng, n, p, lo=1, hi=100, dtype="i32"):
    if dtype == "i32":
        W = np.where(rng.random((n, n)) < p, rng.integers(lo, hi + 1, (n, n)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
    else:
        W = np.where(rng.random((n, n)) < p, rng.uniform(0.1, 10.0, (n, n)), np.inf).astype(np.float32)
        np.fill_diagonal(W, 0.0)
    return W


def test_batched_edge_sizes(native, dev):
    rng = np.random.default_rng(900)
    sizes = [0, 1, 2, 3, 31, 127, 128, 129, 200, 255, 256, 257, 511, 512, 513, 1000, 1024, 5]
    mats = [rand_graph(rng, n, min(0.5, 3.0 / max(n, 1))) for n in sizes]
    sub = native.make_opts(batch_queue=True, tile=64)
    sub.reserved[0] = 128
    for kw in ({}, {"batch_lockstep": True}, {"batch_lockstep": True, "batch_graph": False}, {"batch_persistent": True},
               {"batch_persistent": True, "batch_graph": False}, {"batch_per_graph": True},
               {"batch_queue": True}, {"batch_queue": True, "batch_graph": False}, {"batch_queue": True, "block": 64},
               {"opts": sub}):
        flat, off_d, sz_d, hs, off = pack(mats, dev)
        flags = kw
        native.apsp_batched(flat, off_d, sz_d, hs, **kw)
        for W, got in zip(mats, unpack(flat, off, hs)):
            np.testing.assert_array_equal(got, oracle.fw_i32(W), err_msg=f"n={W.shape[0]} {flags}")
        assert native.apsp_batched_status() == 0, flags


SCHEDS = {"auto": {}, "lockstep": {"batch_lockstep": True}, "persistent": {"batch_persistent": True},
          "queue": {"batch_queue": True}, "queue_sub": {"batch_queue": True, "tile": 64}}


@pytest.mark.parametrize("sched", list(SCHEDS))
def test_batched_f32(native, dev, sched):
    rng = np.random.default_rng(901)
    mats = [rand_graph(rng, n, 4.0 / n, dtype="f32") for n in (40, 130, 300, 77)]
    flat, off_d, sz_d, hs, off = pack(mats, dev)
    native.apsp_batched(flat, off_d, sz_d, hs, **SCHEDS[sched])
    for W, got in zip(mats, unpack(flat, off, hs)):
        ref = oracle.fw_f64(W.astype(np.float64))
        assert np.array_equal(np.isinf(got), np.isinf(ref))
        fin = np.isfinite(ref)
        assert (np.abs(got[fin] - ref[fin]) <= 1e-5 * ref[fin]).all()


@pytest.mark.parametrize("sched", list(SCHEDS))
def test_batched_graph_replays_and_buffer_swaps(native, dev, sched):
    # the captured launch is replayed several times, on two different buffers,
    # with unrelated eager work and synchronisations in between
    rng = np.random.default_rng(902)
    mats = [rand_graph(rng, n, 0.05) for n in (64, 300, 129, 513, 33)]
    refs = [oracle.fw_i32(W) for W in mats]
    bufs = [pack(mats, dev) for _ in range(2)]
    for rep in range(4):
        flat, off_d, sz_d, hs, off = bufs[rep % 2]
        flat.copy_(torch.from_numpy(gg.pack_batch(mats)[0]).to(dev))
        native.apsp_batched(flat, off_d, sz_d, hs, **SCHEDS[sched])
        junk = torch.arange(1000, device=dev).sum()   # eager work between replays
        torch.cuda.synchronize()
        assert int(junk) == 499500
        for ref, got in zip(refs, unpack(flat, off, hs)):
            np.testing.assert_array_equal(got, ref, err_msg=f"replay {rep}")


def test_batched_one_launch_plans_and_plan_switches(native, dev):
    # every graph n <= 128: the lock-step plan is one closure launch, issued
    # directly; alternating it with a multi-launch batch on the same context
    # switches between the direct launch and the captured graph
    rng = np.random.default_rng(903)
    small = [rand_graph(rng, n, min(0.5, 4.0 / max(n, 1))) for n in (0, 1, 2, 17, 64, 100, 127, 128, 5)]
    mixed = [rand_graph(rng, n, 0.05) for n in (90, 300, 129, 40)]
    cases = [(small, [oracle.fw_i32(W) for W in small]), (mixed, [oracle.fw_i32(W) for W in mixed])]
    bufs = {id(m): [pack(m, dev) for _ in range(2)] for m, _ in cases}
    for rep in range(6):
        mats, refs = cases[rep % 2]
        flat, off_d, sz_d, hs, off = bufs[id(mats)][(rep // 2) % 2]
        flat.copy_(torch.from_numpy(gg.pack_batch(mats)[0]).to(dev))
        native.apsp_batched(flat, off_d, sz_d, hs, batch_lockstep=True)
        for ref, got in zip(refs, unpack(flat, off, hs)):
            np.testing.assert_array_equal(got, ref, err_msg=f"call {rep}")


@pytest.mark.parametrize("sched", list(SCHEDS))
def test_batched_workload_512(native, dev, sched):
    batch = gg.batch_ragged()
    mats = [gg.batch_graph_i32(b) for b in batch]
    flat, off_d, sz_d, hs, off = pack(mats, dev)
    native.apsp_batched(flat, off_d, sz_d, hs, **SCHEDS[sched])
    assert native.apsp_batched_status() == 0
    got = unpack(flat, off, hs)
    for b, W, g in zip(batch, mats, got):
        np.testing.assert_array_equal(g, oracle.fw_i32(W, threads=8), err_msg=f"graph {b.g} n={b.n}")


def test_batched_size_limits(native, dev):
    """The lock-step and persistent schedules take n <= 1024, the queue
    schedule (and the automatic plan, which then picks a queue) n <= 8192."""
    W = np.zeros((1025, 1025), np.int32)
    flat, off_d, sz_d, hs, off = pack([W], dev)
    for kw in ({"batch_lockstep": True}, {"batch_persistent": True}):
        with pytest.raises(native.ApspError) as e:
            native.apsp_batched(flat, off_d, sz_d, hs, **kw)
        assert e.value.status == native.APSP_E_UNSUPPORTED
    native.apsp_batched(flat, off_d, sz_d, hs)
    assert native.apsp_batch_candidate(native.apsp_batched_choice()).flags & native.FLAG_BATCH_QUEUE
    big = torch.zeros(8193 * 8193, dtype=torch.int32, device=dev)
    with pytest.raises(native.ApspError) as e:
        native.apsp_batched(big, torch.zeros(1, dtype=torch.int64, device=dev),
                            torch.full((1,), 8193, dtype=torch.int32, device=dev), [8193], batch_queue=True)
    assert e.value.status == native.APSP_E_UNSUPPORTED


GLOBAL_CASES = [(1500, 0.01, {"batch_queue": True, "batch_global": True}),
                (2500, 0.004, {"batch_queue": True, "batch_global": True, "block": 128, "tile": 64}),
                (1200, 0.02, {"batch_queue": True, "batch_global": True, "block": 64}),
                (2049, 0.003, {})]


@pytest.mark.parametrize("n,p,kw", GLOBAL_CASES, ids=[f"n{n}_{i}" for i, (n, p, kw) in enumerate(GLOBAL_CASES)])
def test_queue_large_single_graph(native, dev, n, p, kw):
    """One graph above the lock-step limit through the queue schedule with
    one queue for the device (its tasks run on every XCD; the automatic plan
    takes this form for a batch of one), bit-exact against the oracle; a
    second graph of other size in the same batch."""
    rng = np.random.default_rng(n)
    mats = []
    for m in (n, 300):
        W = np.where(rng.random((m, m)) < p * (n / m), rng.integers(1, 1000, (m, m)), INF).astype(np.int32)
        np.fill_diagonal(W, 0)
        mats.append(W)
    flat, off_d, sz_d, hs, off = pack(mats, dev)
    native.apsp_batched(flat, off_d, sz_d, hs, **kw)
    assert native.apsp_batched_status() == 0
    got = unpack(flat, off, hs)
    for W, g in zip(mats, got):
        np.testing.assert_array_equal(g, oracle.fw_i32(W, threads=16), err_msg=f"n={W.shape[0]} {kw}")


def test_batched_workspace_contract(native, dev):
    """apsp_batched keeps its plan in the caller's workspace: without one, or
    with one smaller than apsp_workspace_size says, it returns APSP_E_NOMEM
    before enqueuing anything (the data stays untouched); a workspace of the
    reported size works, also after a predecessor call reused it and after
    the workspace was replaced."""
    import ctypes
    rng = np.random.default_rng(940)
    mats = [rand_graph(rng, n, 4.0 / n) for n in (300, 40, 512, 129, 64)]
    refs = [oracle.fw_i32(W) for W in mats]
    L = native.lib()
    ctx = native.context(dev.index)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    saved = native._ws.get(dev.index)

    def call():
        flat, off_d, sz_d, hs, off = pack(mats, dev)
        before = flat.clone()
        h = (ctypes.c_int32 * len(hs))(*hs)
        o = native.make_opts()
        rc = L.apsp_batched(ctx, 0, len(hs), flat.data_ptr(), off_d.data_ptr(), sz_d.data_ptr(), h,
                            ctypes.byref(o), st)
        return rc, flat, before, off, hs

    try:
        need = native.apsp_workspace_size("batched", 512, len(mats))
        assert need > 0
        native.apsp_set_workspace(None, dev.index)
        rc, flat, before, _, _ = call()
        assert rc == native.APSP_E_NOMEM and "workspace" in native.last_error()
        torch.cuda.synchronize()
        assert torch.equal(flat, before)
        native.apsp_set_workspace(torch.empty(1024, dtype=torch.uint8, device=dev), dev.index)
        rc, flat, before, _, _ = call()
        assert rc == native.APSP_E_NOMEM
        torch.cuda.synchronize()
        assert torch.equal(flat, before)
        for _ in range(2):
            native.apsp_set_workspace(torch.empty(need, dtype=torch.uint8, device=dev), dev.index)
            rc, flat, _, off, hs = call()
            assert rc == native.APSP_OK
            for ref, got in zip(refs, unpack(flat, off, hs)):
                np.testing.assert_array_equal(got, ref)
            # another user of the workspace in between: the plan is uploaded again
            W = mats[0]
            Dd = torch.from_numpy(refs[0]).to(dev)
            native.apsp_predecessors(Dd, torch.from_numpy(W).to(dev), method="sparse")
            rc, flat, _, off, hs = call()
            assert rc == native.APSP_OK
            for ref, got in zip(refs, unpack(flat, off, hs)):
                np.testing.assert_array_equal(got, ref)
    finally:
        native.apsp_set_workspace(saved, dev.index)
