"""Python binding of libapsp (include/apsp.h): argument marshalling only.

Every function here has the name of the C entry point it calls and forwards
device pointers, leading dimensions and torch's current HIP stream; all
arithmetic happens in the HIP kernels behind the C ABI.  torch is used only
for device memory and streams.  If libapsp.so has not been built the import
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libapsp.so")

APSP_OK, APSP_E_ARG, APSP_E_INPUT, APSP_E_NOMEM, APSP_E_HIP, APSP_E_UNSUPPORTED, APSP_E_STATE = 0, -1, -2, -3, -4, -5, -6
APSP_I32, APSP_F32 = 0, 1
INF_I32 = 1 << 30
ALGO = {"auto": 0, "fw": 1, "rkleene": 2, "square": 3}
CLOSURE = {"auto": 0, "kloop": 1, "square": 2}
TILE = {"auto": 0, 128: 1, 64: 2}
FLAG_NO_SPLITK, FLAG_BATCH_NO_GRAPH, FLAG_BATCH_PER_GRAPH, FLAG_NO_LOOKAHEAD, FLAG_BATCH_PERSISTENT = 1, 2, 4, 8, 16
FLAG_PACKED16 = 32
FLAG_SKIP_INF = 64
FLAG_BATCH_QUEUE = 128
FLAG_BATCH_LOCKSTEP = 256
FLAG_BATCH_GLOBAL = 512
FLAG_DETERMINISTIC = 1024
CAP16 = 0x39FF    # 14847: cap of the APSP_FLAG_PACKED16 products

# every symbol include/apsp.h declares
EXPORTS = [
    "apsp_create", "apsp_destroy", "apsp_last_error", "apsp_version",
    "minplus_gemm", "apsp_closure", "apsp_fw", "apsp_rkleene", "apsp_square",
    "apsp_solve", "apsp_batched", "apsp_validate", "apsp_profile_enable", "apsp_profile_read",
    "apsp_candidate_count", "apsp_candidate", "apsp_costmodel_init", "apsp_costmodel_set_norm",
    "apsp_costmodel_set_params", "apsp_costmodel_get_params", "apsp_costmodel_save", "apsp_costmodel_load",
    "apsp_costmodel_train", "apsp_costmodel_grad",
    "apsp_costmodel_forward", "apsp_costmodel_predict", "apsp_plan", "apsp_predecessors",
    "apsp_packed16_counts", "apsp_predecessors_ex", "apsp_measure_fold_rate",
    "apsp_workspace_size", "apsp_set_workspace", "apsp_path", "apsp_batched_noalloc",
    "apsp_features", "apsp_solve_choice", "apsp_batched_status",
    "apsp_batch_candidate_count", "apsp_batch_candidate", "apsp_plan_batch", "apsp_batched_choice",
    "apsp_square_passes",
]
# the trained cost model shipped with the package (plain-text model file)
MODEL_PATH = os.path.join(_PKG, "data", "costmodel_mlp.txt")
OP = {"solve": 0, "batched": 1, "predecessors": 2, "deterministic": 3}
FOLD = {"int32": 0, "float32": 1, "packed16": 2}
PRED = {"auto": 0, "dense": 1, "sparse": 2}

KERNEL_MINPLUS_128, KERNEL_MINPLUS_64, KERNEL_CLOSURE, KERNEL_OTHER = 0, 1, 2, 3


class ApspError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


class Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("block", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("closure", ctypes.c_int32), ("cutover", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("reserved", ctypes.c_int32 * 3)]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("milliseconds", ctypes.c_double),
                ("terms", ctypes.c_double), ("bytes", ctypes.c_double)]


def make_opts(algo="auto", block=0, tile="auto", closure="auto", cutover=0, splitk=True,
              batch_graph=True, batch_per_graph=False, lookahead=True, batch_persistent=False,
              packed16=False, skip_inf=False, batch_queue=False, batch_lockstep=False,
              batch_global=False, deterministic=False) -> Opts:
    o = Opts()
    o.algo = ALGO[algo] if isinstance(algo, str) else int(algo)
    o.block = int(block)
    o.tile = TILE[tile]
    o.closure = CLOSURE[closure] if isinstance(closure, str) else int(closure)
    o.cutover = int(cutover)
    o.flags = (0 if splitk else FLAG_NO_SPLITK) | (0 if batch_graph else FLAG_BATCH_NO_GRAPH) | \
        (FLAG_BATCH_PER_GRAPH if batch_per_graph else 0) | (0 if lookahead else FLAG_NO_LOOKAHEAD) | \
        (FLAG_BATCH_PERSISTENT if batch_persistent else 0) | (FLAG_PACKED16 if packed16 else 0) | \
        (FLAG_SKIP_INF if skip_inf else 0) | (FLAG_BATCH_QUEUE if batch_queue else 0) | \
        (FLAG_BATCH_LOCKSTEP if batch_lockstep else 0) | (FLAG_BATCH_GLOBAL if batch_global else 0) | \
        (FLAG_DETERMINISTIC if deterministic else 0)
    return o


_lock = threading.Lock()
_lib = None
_ctxs: dict[int, ctypes.c_void_p] = {}
_ws: dict[int, torch.Tensor] = {}     # workspace registered with each device's context


def lib() -> ctypes.CDLL:
    """Loads libapsp.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2310_03983_amd.build` (there is no CPU fallback)")
            L = ctypes.CDLL(LIB_PATH)
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            P = ctypes.POINTER
            L.apsp_create.argtypes = [P(vp), i32]
            L.apsp_destroy.argtypes = [vp]
            L.apsp_last_error.restype = ctypes.c_char_p
            L.apsp_last_error.argtypes = []
            L.apsp_version.restype = ctypes.c_char_p
            L.apsp_version.argtypes = []
            L.minplus_gemm.argtypes = [vp, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, P(Opts), vp]
            for name in ("apsp_closure", "apsp_fw", "apsp_rkleene", "apsp_square", "apsp_solve"):
                getattr(L, name).argtypes = [vp, i32, i64, vp, i64, P(Opts), vp]
            L.apsp_batched.argtypes = [vp, i32, i32, vp, vp, vp, P(i32), P(Opts), vp]
            L.apsp_batched_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, P(i32), P(Opts), vp]
            L.apsp_validate.argtypes = [vp, i32, i64, vp, i64, vp, P(i64)]
            L.apsp_predecessors.argtypes = [vp, i32, i64, vp, i64, vp, i64, vp, i64, vp]
            L.apsp_predecessors_ex.argtypes = [vp, i32, i64, vp, i64, vp, i64, vp, i64, i32, vp]
            L.apsp_profile_enable.argtypes = [vp, i32]
            L.apsp_profile_read.argtypes = [vp, i32, P(KernelStats)]
            f32p = P(ctypes.c_float)
            L.apsp_candidate_count.argtypes = []
            L.apsp_candidate.argtypes = [i32, P(Opts)]
            L.apsp_costmodel_init.argtypes = [vp, i32, ctypes.c_uint64]
            L.apsp_costmodel_set_norm.argtypes = [vp, f32p, f32p]
            L.apsp_costmodel_set_params.argtypes = [vp, f32p, i64]
            L.apsp_costmodel_get_params.argtypes = [vp, f32p, i64]
            L.apsp_measure_fold_rate.argtypes = [vp, i32, vp, P(ctypes.c_double), P(ctypes.c_double)]
            L.apsp_costmodel_save.argtypes = [vp, ctypes.c_char_p]
            L.apsp_costmodel_load.argtypes = [vp, ctypes.c_char_p]
            L.apsp_costmodel_train.argtypes = [vp, vp, vp, vp, i32, P(TrainCfg), vp, vp]
            L.apsp_costmodel_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
            L.apsp_costmodel_forward.argtypes = [vp, vp, i32, vp, vp]
            L.apsp_costmodel_predict.argtypes = [vp, vp, i32, vp, vp]
            L.apsp_plan.argtypes = [vp, i32, i64, ctypes.c_double, i32, i32, P(Opts), P(i32)]
            L.apsp_workspace_size.argtypes = [vp, i32, i32, i64, i32]
            L.apsp_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
            L.apsp_path.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp, i32, vp, vp]
            L.apsp_features.argtypes = [vp, i32, i64, vp, i64, vp, P(ctypes.c_float)]
            L.apsp_solve_choice.argtypes = [vp, P(i32)]
            L.apsp_square_passes.argtypes = [vp, vp, P(i32)]
            L.apsp_batched_status.argtypes = [vp, vp, P(ctypes.c_uint32)]
            L.apsp_batch_candidate_count.argtypes = []
            L.apsp_batch_candidate.argtypes = [i32, P(Opts)]
            L.apsp_plan_batch.argtypes = [vp, i32, i32, P(i32), ctypes.c_double, P(Opts), P(i32)]
            L.apsp_batched_choice.argtypes = [vp, P(i32)]
            for name in EXPORTS:
                if name not in ("apsp_last_error", "apsp_version", "apsp_workspace_size"):
                    getattr(L, name).restype = i32
            L.apsp_workspace_size.restype = ctypes.c_size_t
            _lib = L
    return _lib


def last_error() -> str:
    return lib().apsp_last_error().decode()


def _check(status: int):
    if status != APSP_OK:
        raise ApspError(status, last_error())


def context(device: int | None = None) -> ctypes.c_void_p:
    """The library context of a HIP device (created once per process)."""
    if device is None:
        device = torch.cuda.current_device()
    with _lock:
        c = _ctxs.get(device)
    if c is None:
        c = ctypes.c_void_p()
        _check(lib().apsp_create(ctypes.byref(c), device))
        with _lock:
            _ctxs[device] = c
        # the shipped cost model plans apsp_solve's automatic choice
        if os.path.exists(MODEL_PATH) and os.environ.get("APSP_NO_MODEL") != "1":
            _check(lib().apsp_costmodel_load(c, os.fsencode(MODEL_PATH)))
    return c


def apsp_workspace_size(op: str, n_or_total: int, count: int = 0, dtype: str = "int32",
                        device: int | None = None) -> int:
    """Bytes of workspace `op` ("solve", "batched", "predecessors") needs."""
    dt = {"int32": APSP_I32, "float32": APSP_F32}[dtype]
    return int(lib().apsp_workspace_size(context(device), OP[op], dt, int(n_or_total), int(count)))


def apsp_set_workspace(buf: torch.Tensor | None, device: int | None = None):
    """Registers a device tensor (any dtype, contiguous) as the context's
    workspace, or clears it with None.  The binding keeps a reference."""
    if device is None:
        device = buf.device.index if buf is not None else torch.cuda.current_device()
    if buf is None:
        _check(lib().apsp_set_workspace(context(device), None, 0))
        _ws.pop(device, None)
        return
    if not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("workspace must be a contiguous device tensor")
    _check(lib().apsp_set_workspace(context(device), buf.data_ptr(), buf.numel() * buf.element_size()))
    _ws[device] = buf


def _ensure_workspace(op: str, dt: int, n_or_total: int, count: int, device: int):
    """Allocates (through torch) and registers a workspace large enough for
    `op` when the registered one is smaller."""
    need = int(lib().apsp_workspace_size(context(device), OP[op], dt, int(n_or_total), int(count)))
    cur = _ws.get(device)
    if need and (cur is None or cur.numel() < need):
        apsp_set_workspace(torch.empty(need, dtype=torch.uint8, device=torch.device("cuda", device)), device)


def _dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return APSP_I32
    if t.dtype == torch.float32:
        return APSP_F32
    raise TypeError(f"dtype {t.dtype} is not supported (int32 or float32)")


def _matrix(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")
    return t.data_ptr(), max(t.stride(0), t.shape[1])


def _stream(t: torch.Tensor, stream):
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(stream.cuda_stream)


def _opts(opts, kw) -> Opts:
    if opts is not None:
        return opts
    return make_opts(**kw)


def minplus_gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, opts: Opts | None = None,
                 stream=None, **kw) -> torch.Tensor:
    """C <- min(C, A (min,+) B) in place (Sec. 3, Eq. 2); returns C."""
    dt = _dtype(C)
    if A.dtype != C.dtype or B.dtype != C.dtype:
        raise TypeError("A, B and C must share a dtype")
    pa, lda = _matrix(A, "A")
    pb, ldb = _matrix(B, "B")
    pc, ldc = _matrix(C, "C")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    o = _opts(opts, kw)
    _check(lib().minplus_gemm(context(C.device.index), dt, m, n, k, pa, lda, pb, ldb, pc, ldc,
                              ctypes.byref(o), _stream(C, stream)))
    return C


def _square_call(name, D, opts, stream, kw):
    dt = _dtype(D)
    p, ld = _matrix(D, "D")
    n = D.shape[0]
    if D.shape[1] != n:
        raise ValueError("D must be square")
    o = _opts(opts, kw)
    if o.flags & FLAG_DETERMINISTIC and name in ("apsp_fw", "apsp_rkleene", "apsp_solve") and D.is_cuda:
        _ensure_workspace("deterministic", dt, n, 0, D.device.index)
    _check(getattr(lib(), name)(context(D.device.index), dt, n, p, ld, ctypes.byref(o), _stream(D, stream)))
    return D


def apsp_closure(D, opts=None, stream=None, **kw):
    """Closure of one block of at most 128 x 128 (Sec. 2, Eq. 1); in place."""
    return _square_call("apsp_closure", D, opts, stream, kw)


def apsp_fw(D, opts=None, stream=None, **kw):
    """Three-phase blocked Floyd-Warshall (Sec. 2, Eq. 1); D is overwritten."""
    return _square_call("apsp_fw", D, opts, stream, kw)


def apsp_rkleene(D, opts=None, stream=None, **kw):
    """R-Kleene quadrant recursion (Sec. 3.3, Eq. 4); D is overwritten."""
    return _square_call("apsp_rkleene", D, opts, stream, kw)


def apsp_square(D, opts=None, stream=None, **kw):
    """Min-plus squaring until unchanged (Sec. 3.2); D is overwritten."""
    return _square_call("apsp_square", D, opts, stream, kw)


def apsp_solve(D, opts=None, stream=None, **kw):
    """Planner-selected algorithm; D is overwritten.  With no options the
    context's cost model plans from the matrix (a workspace for the feature
    pass is registered first)."""
    if opts is None and not kw and D.is_cuda:
        _ensure_workspace("solve", _dtype(D), D.shape[0], 0, D.device.index)
    return _square_call("apsp_solve", D, opts, stream, kw)


def apsp_solve_choice(device: int | None = None) -> int:
    """Candidate index the last automatic apsp_solve ran (-1: size rule)."""
    ch = ctypes.c_int32(-1)
    _check(lib().apsp_solve_choice(context(device), ctypes.byref(ch)))
    return int(ch.value)


def apsp_features(D, stream=None) -> list[float]:
    """The cost model's four inputs for the cost matrix D, computed on the
    device (log2 n, log10 density, log2 batch = 0, weakly connected)."""
    dt = _dtype(D)
    p, ld = _matrix(D, "D")
    n = D.shape[0]
    _ensure_workspace("solve", dt, n, 0, D.device.index)
    out = (ctypes.c_float * 4)()
    _check(lib().apsp_features(context(D.device.index), dt, n, p, ld, _stream(D, stream), out))
    return [float(v) for v in out]


def apsp_predecessors(D, W, P=None, stream=None, method="auto"):
    """Last-hop predecessor matrix (int32 device tensor) of distances D for
    costs W (Sec. 2); allocates P when it is not given.  method: "auto",
    "dense" or "sparse" (apsp_predecessors_ex)."""
    dt = _dtype(D)
    if W.dtype != D.dtype:
        raise TypeError("D and W must share a dtype")
    pd, ldd = _matrix(D, "D")
    pw, ldw = _matrix(W, "W")
    n = D.shape[0]
    if tuple(D.shape) != (n, n) or tuple(W.shape) != (n, n):
        raise ValueError("D and W must be n x n")
    if P is None:
        P = torch.empty((n, n), dtype=torch.int32, device=D.device)
    if P.dtype != torch.int32:
        raise TypeError("P must be int32")
    pp, ldp = _matrix(P, "P")
    if method != "dense":
        _ensure_workspace("predecessors", dt, n, 0, D.device.index)
    _check(lib().apsp_predecessors_ex(context(D.device.index), dt, n, pd, ldd, pw, ldw, pp, ldp, PRED[method],
                                      _stream(D, stream)))
    return P


def apsp_path(P: torch.Tensor, src, dst, max_len: int | None = None, stream=None) -> list[list[int]]:
    """Vertices of the src[q] -> dst[q] paths encoded by the predecessor
    matrix P (apsp_path; Sec. 2): one list per query, source first, [] when
    the target is unreachable.  src and dst are ints or equal-length
    sequences.  Raises ValueError for a broken chain."""
    if P.dtype != torch.int32:
        raise TypeError("P must be int32")
    pp, ldp = _matrix(P, "P")
    n = P.shape[0]
    single = isinstance(src, int) and isinstance(dst, int)
    s_ = [int(src)] if single else [int(x) for x in src]
    d_ = [int(dst)] if single else [int(x) for x in dst]
    if len(s_) != len(d_):
        raise ValueError("src and dst differ in length")
    count = len(s_)
    L = int(max_len or max(n, 1))
    dev = P.device
    sd = torch.tensor(s_, dtype=torch.int32, device=dev)
    dd = torch.tensor(d_, dtype=torch.int32, device=dev)
    paths = torch.empty((max(count, 1), L), dtype=torch.int32, device=dev)
    lens = torch.empty(max(count, 1), dtype=torch.int32, device=dev)
    _check(lib().apsp_path(context(dev.index), n, pp, ldp, count, sd.data_ptr(), dd.data_ptr(), paths.data_ptr(), L,
                           lens.data_ptr(), _stream(P, stream)))
    lh = lens.cpu().tolist()
    ph = paths.cpu()
    out = []
    for q in range(count):
        if lh[q] < 0:
            raise ValueError(f"broken predecessor chain for {s_[q]} -> {d_[q]}")
        out.append(ph[q, :lh[q]].tolist())
    return out[0] if single else out


def apsp_validate(D, stream=None) -> int:
    """Number of entries violating the input contract (synchronous)."""
    dt = _dtype(D)
    p, ld = _matrix(D, "D")
    n = D.shape[0]
    v = ctypes.c_int64(0)
    st = lib().apsp_validate(context(D.device.index), dt, n, p, ld, _stream(D, stream), ctypes.byref(v))
    if st not in (APSP_OK, APSP_E_INPUT):
        _check(st)
    return int(v.value)


def apsp_batched(data: torch.Tensor, offsets: torch.Tensor, sizes: torch.Tensor, h_sizes,
                 opts=None, stream=None, **kw):
    """Closes every graph of a ragged batch in one launch; `data` is overwritten."""
    dt = _dtype(data)
    if not (data.is_cuda and offsets.is_cuda and sizes.is_cuda):
        raise TypeError("data, offsets and sizes must be device tensors")
    if offsets.dtype != torch.int64 or sizes.dtype != torch.int32:
        raise TypeError("offsets must be int64 and sizes int32")
    count = len(h_sizes)
    hs = (ctypes.c_int32 * max(count, 1))(*[int(x) for x in h_sizes])
    o = _opts(opts, kw)
    if count:
        _ensure_workspace("batched", dt, max(int(x) for x in h_sizes), count, data.device.index)
    _check(lib().apsp_batched(context(data.device.index), dt, count, data.data_ptr(), offsets.data_ptr(),
                              sizes.data_ptr(), hs, ctypes.byref(o), _stream(data, stream)))
    return data


def apsp_batched_noalloc(data: torch.Tensor, offsets: torch.Tensor, sizes: torch.Tensor, h_sizes,
                         opts=None, stream=None, **kw):
    """apsp_batched with the plan in the library's fixed device array: no
    workspace, nothing allocated; `data` is overwritten."""
    dt = _dtype(data)
    if not (data.is_cuda and offsets.is_cuda and sizes.is_cuda):
        raise TypeError("data, offsets and sizes must be device tensors")
    if offsets.dtype != torch.int64 or sizes.dtype != torch.int32:
        raise TypeError("offsets must be int64 and sizes int32")
    count = len(h_sizes)
    hs = (ctypes.c_int32 * max(count, 1))(*[int(x) for x in h_sizes])
    o = _opts(opts, kw)
    _check(lib().apsp_batched_noalloc(context(data.device.index), dt, count, data.data_ptr(), offsets.data_ptr(),
                                      sizes.data_ptr(), hs, ctypes.byref(o), _stream(data, stream)))
    return data


def apsp_batched_status(device: int | None = None) -> int:
    """Error word of the last batched plan (bit 0: a queue wait overran),
    cleared by the call."""
    dev = torch.cuda.current_device() if device is None else device
    f = ctypes.c_uint32(0)
    _check(lib().apsp_batched_status(context(dev), ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                     ctypes.byref(f)))
    return int(f.value)


def apsp_profile_enable(on: bool = True, kinds=None, device: int | None = None):
    """Starts (clearing old records) or stops per-launch event timing; with
    `kinds` (iterable of KERNEL_*) only those kernels are bracketed."""
    if not on:
        flag = 0
    elif kinds is None:
        flag = 1
    else:
        flag = 0
        for k in kinds:
            flag |= 1 << k
        if flag == 1:          # only kind 0: 1 would mean "all kinds"
            flag = 1 | (1 << 31)
    _check(lib().apsp_profile_enable(context(device), flag))


def apsp_profile_read(kind: int, device: int | None = None) -> dict:
    """Per-kind launch count, summed milliseconds, min-plus terms and bytes."""
    st = KernelStats()
    _check(lib().apsp_profile_read(context(device), kind, ctypes.byref(st)))
    return {"launches": st.launches, "ms": st.milliseconds, "terms": st.terms, "bytes": st.bytes}


def apsp_square_passes(device: int | None = None) -> int:
    """Passes the last apsp_square on this device's context ran (waits for
    torch's current stream after the one-launch form)."""
    dev = torch.cuda.current_device() if device is None else device
    p = ctypes.c_int32(0)
    _check(lib().apsp_square_passes(context(dev), ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                    ctypes.byref(p)))
    return int(p.value)


def apsp_packed16_counts(device: int | None = None) -> tuple[int, int]:
    """(solves run with packed16=True, how many of them were redone in int32)."""
    runs, redone = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().apsp_packed16_counts(context(device), ctypes.byref(runs), ctypes.byref(redone)))
    return runs.value, redone.value


# ---------------------------------------------------------------------------
# candidate plans and the cost model
# ---------------------------------------------------------------------------

def apsp_candidate_count() -> int:
    return int(lib().apsp_candidate_count())


def apsp_candidate(index: int) -> Opts:
    o = Opts()
    _check(lib().apsp_candidate(index, ctypes.byref(o)))
    return o


def apsp_batch_candidate_count() -> int:
    return int(lib().apsp_batch_candidate_count())


def apsp_batch_candidate(index: int) -> Opts:
    o = Opts()
    _check(lib().apsp_batch_candidate(index, ctypes.byref(o)))
    return o


def apsp_plan_batch(h_sizes, density: float, dtype: str = "int32", device: int | None = None):
    """(Opts, batch candidate index or -1 for the default) for a batch of the
    given sizes and density (apsp_plan_batch)."""
    o = Opts()
    ch = ctypes.c_int32(-1)
    hs = (ctypes.c_int32 * max(len(h_sizes), 1))(*[int(x) for x in h_sizes])
    _check(lib().apsp_plan_batch(context(device), {"int32": 0, "float32": 1}[dtype], len(h_sizes), hs,
                                 float(density), ctypes.byref(o), ctypes.byref(ch)))
    return o, int(ch.value)


def apsp_batched_choice(device: int | None = None) -> int:
    """Batch candidate the last automatic apsp_batched plan chose (-1: none)."""
    ch = ctypes.c_int32(-1)
    _check(lib().apsp_batched_choice(context(device), ctypes.byref(ch)))
    return int(ch.value)


def mlp_param_count(K: int) -> int:
    return 4 * 64 + 64 + 64 * 64 + 64 + 64 * K + K


def _f32_dev(t: torch.Tensor, name: str):
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return t.data_ptr()


def apsp_costmodel_init(K: int, seed: int = 0, device: int | None = None):
    _check(lib().apsp_costmodel_init(context(device), K, seed))


def apsp_costmodel_set_norm(mu, sd, device: int | None = None):
    m = (ctypes.c_float * 4)(*[float(x) for x in mu])
    s_ = (ctypes.c_float * 4)(*[float(x) for x in sd])
    _check(lib().apsp_costmodel_set_norm(context(device), m, s_))


def apsp_costmodel_set_params(params, device: int | None = None):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().apsp_costmodel_set_params(context(device), a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))


def apsp_costmodel_get_params(K: int, device: int | None = None):
    import numpy as np
    a = np.empty(mlp_param_count(K), dtype=np.float32)
    _check(lib().apsp_costmodel_get_params(context(device), a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


def apsp_measure_fold_rate(fold: str = "int32", device: int | None = None, stream=None) -> dict:
    """Spin-kernel issue rate of a fold ("int32", "float32", "packed16"):
    {"terms_per_s", "lane_instr_per_s"} (apsp_measure_fold_rate)."""
    t, li = ctypes.c_double(0.0), ctypes.c_double(0.0)
    dev = torch.cuda.current_device() if device is None else device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib().apsp_measure_fold_rate(context(dev), FOLD[fold], ctypes.c_void_p(st.cuda_stream),
                                        ctypes.byref(t), ctypes.byref(li)))
    return {"terms_per_s": t.value, "lane_instr_per_s": li.value}


def apsp_costmodel_save(path, device: int | None = None):
    """Writes the context's model to a text file (apsp_costmodel_save)."""
    _check(lib().apsp_costmodel_save(context(device), os.fsencode(path)))


def apsp_costmodel_load(path, device: int | None = None):
    """Reads a model file into the context (apsp_costmodel_load)."""
    _check(lib().apsp_costmodel_load(context(device), os.fsencode(path)))


def apsp_costmodel_train(X, T, mask, steps=500, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, losses=None, stream=None):
    cfg = TrainCfg(steps, lr, beta1, beta2, eps)
    lp = _f32_dev(losses, "losses") if losses is not None else None
    _check(lib().apsp_costmodel_train(context(X.device.index), _f32_dev(X, "X"), _f32_dev(T, "T"),
                                      _f32_dev(mask, "mask"), X.shape[0], ctypes.byref(cfg), lp, _stream(X, stream)))


def apsp_costmodel_grad(X, T, mask, grad, loss=None, stream=None):
    lp = _f32_dev(loss, "loss") if loss is not None else None
    _check(lib().apsp_costmodel_grad(context(X.device.index), _f32_dev(X, "X"), _f32_dev(T, "T"),
                                     _f32_dev(mask, "mask"), X.shape[0], _f32_dev(grad, "grad"), lp,
                                     _stream(X, stream)))


def apsp_costmodel_forward(X, out, stream=None):
    _check(lib().apsp_costmodel_forward(context(X.device.index), _f32_dev(X, "X"), X.shape[0],
                                        _f32_dev(out, "out"), _stream(X, stream)))
    return out


def apsp_costmodel_predict(X, choice, stream=None):
    if not choice.is_cuda or choice.dtype != torch.int32:
        raise TypeError("choice must be an int32 device tensor")
    _check(lib().apsp_costmodel_predict(context(X.device.index), _f32_dev(X, "X"), X.shape[0],
                                        choice.data_ptr(), _stream(X, stream)))
    return choice


def apsp_plan(n: int, density: float, batch: int = 1, connected: bool = True, dtype: str = "int32",
              device: int | None = None):
    """Returns (Opts, candidate index or -1 for the built-in size rule) for a
    problem of `dtype` ("int32" or "float32")."""
    o = Opts()
    ch = ctypes.c_int32(-1)
    dt = {"int32": 0, "float32": 1}[dtype]
    _check(lib().apsp_plan(context(device), dt, n, float(density), batch, 1 if connected else 0,
                           ctypes.byref(o), ctypes.byref(ch)))
    return o, int(ch.value)
