"""apsp_batched_noalloc (plan in the library's fixed device array, nothing
allocated) against apsp_batched (plan in the caller's workspace) through the
C ABI: bit-identical int32 results on two calls in a row, the second with a
smaller batch, both schedules; every graph also against the oracle; a batch
whose plan exceeds the fixed array is rejected before anything runs."""
import ctypes

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


def run(native, fn_name, mats, dev, flags=0):
    flat, off, sz = gg.pack_batch(mats)
    data = torch.from_numpy(flat).to(dev)
    off_d = torch.from_numpy(off).to(dev)
    sz_d = torch.from_numpy(sz).to(dev)
    hs = (ctypes.c_int32 * len(mats))(*[int(m.shape[0]) for m in mats])
    o = native.make_opts()
    o.flags = flags
    if fn_name == "apsp_batched":
        native._ensure_workspace("batched", 0, max(int(m.shape[0]) for m in mats), len(mats), dev.index)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(native.lib(), fn_name)(native.context(dev.index), 0, len(mats), data.data_ptr(), off_d.data_ptr(),
                                        sz_d.data_ptr(), hs, ctypes.byref(o), st)
    assert rc == native.APSP_OK, native.last_error()
    torch.cuda.synchronize()
    h = data.cpu().numpy()
    return [h[o_:o_ + m.shape[0] ** 2].reshape(m.shape) for o_, m in zip(off, mats)]


@pytest.mark.parametrize("flags", [0, 16])   # lock-step, persistent
def test_noalloc_matches_batched(native, dev, flags):
    rng = np.random.default_rng(7000 + flags)
    first = [rand_graph(rng, n, min(0.5, 4.0 / max(n, 1))) for n in (512, 300, 129, 64, 33, 1, 0, 200, 511, 128)]
    second = [rand_graph(rng, n, min(0.5, 4.0 / max(n, 1))) for n in (260, 17, 100)]
    for mats in (first, second):
        want = run(native, "apsp_batched", mats, dev, flags)
        got = run(native, "apsp_batched_noalloc", mats, dev, flags)
        for W, a, b in zip(mats, want, got):
            np.testing.assert_array_equal(b, a, err_msg=f"n={W.shape[0]}")
            np.testing.assert_array_equal(b, oracle.fw_i32(W), err_msg=f"n={W.shape[0]}")


def test_noalloc_rejects_oversized_plan(native, dev):
    """4000 graphs of n = 512 need 640 000 work items (160 each: one closure,
    then per 128-wide round 6 panel tiles, the next pivot and 32 or 36
    remainder sub-tiles), 10.2 MB of plan, more than the 8 MiB array.  The
    buffers are real (empty graphs), so a call that ran anyway would stay in
    bounds; it must be rejected before anything is enqueued."""
    count, n = 4000, 512
    data = torch.full((count * n * n,), INF, dtype=torch.int32, device=dev)
    off = torch.arange(count, dtype=torch.int64, device=dev) * (n * n)
    sz = torch.full((count,), n, dtype=torch.int32, device=dev)
    hs = (ctypes.c_int32 * count)(*([n] * count))
    o = native.make_opts()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = native.lib().apsp_batched_noalloc(native.context(dev.index), 0, count, data.data_ptr(), off.data_ptr(),
                                           sz.data_ptr(), hs, ctypes.byref(o), st)
    assert rc == native.APSP_E_UNSUPPORTED
    assert "fixed scratch" in native.last_error()
    torch.cuda.synchronize()
    assert bool((data == INF).all())
