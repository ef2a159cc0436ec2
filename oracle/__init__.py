"""CPU oracle for min-plus APSP -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library
(``paper_2310_03983_amd``) never imports, links or calls it, and this package
imports nothing from the product: the two share no code.  Seeded inputs come
from ``paper_2310_03983_amd.graphgen``, which holds no APSP arithmetic; the
tests pass the same arrays to both sides.

Contents (paper: arXiv 2310.03983, "The Floyd-Warshall Algorithm
Re-implemented Using 3D-Tensors and Hardware Acceleration"):

* ``fw_i32`` / ``fw_f64``         -- triple-loop Floyd-Warshall, Sec. 2 Eq. 1 (C).
* ``fw_i32_steps``                -- passes k0 .. k1-1 of that loop (C); a bounded
  sample for timing, pinned by the restricted-intermediate invariant.
* ``minplus_i32`` / ``minplus_f32`` -- accumulating min-plus product, Sec. 3
  Eq. 2 (C): ``C <- min(C, A (min,+) B)``.
* ``dijkstra_i32`` / ``dijkstra_f64`` -- per-source Dijkstra (C); an algorithm
  independent of Eq. 1 used to cross-check it and to sample large results.
* ``certificate_i32``             -- Bellman optimality certificate (C).
* ``brute_apsp``                   -- exhaustive simple-path enumeration (Python).
* ``bfs_hops``                     -- BFS hop counts for unit weights (Python).
* ``mlp_*``                        -- fp64 numpy reference of the cost-model MLP
  (forward, masked-MSE loss, backward, Adam step).

INF conventions: int32 ``INF = 2**30`` with saturating addition
``a (+) b = min(a + b, INF)``; floating point ``INF = +inf``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

INF_I32 = 1 << 30

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP for the per-source and
    per-row loops only).  Returns the path of the shared library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
            lib.oracle_fw_i32.argtypes = [i64, vp, i64, i32]
            lib.oracle_fw_i32.restype = None
            lib.oracle_fw_i32_steps.argtypes = [i64, vp, i64, i64, i64, i32]
            lib.oracle_fw_i32_steps.restype = None
            lib.oracle_fw_f64.argtypes = [i64, vp, i64, i32]
            lib.oracle_fw_f64.restype = None
            lib.oracle_minplus_i32.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
            lib.oracle_minplus_i32.restype = None
            lib.oracle_minplus_f32.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
            lib.oracle_minplus_f32.restype = None
            lib.oracle_dijkstra_i32.argtypes = [i64, vp, i64, i64, vp, vp, i32]
            lib.oracle_dijkstra_i32.restype = i32
            lib.oracle_dijkstra_f64.argtypes = [i64, vp, i64, i64, vp, vp, i32]
            lib.oracle_dijkstra_f64.restype = i32
            lib.oracle_certificate_i32.argtypes = [i64, vp, i64, vp, i64, i64, i64, i32]
            lib.oracle_certificate_i32.restype = i64
            lib.oracle_predecessors_i32.argtypes = [i64, vp, i64, vp, i64, vp, i64, i32]
            lib.oracle_predecessors_i32.restype = None
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def default_threads() -> int:
    """The host threads the oracle uses: OMP_NUM_THREADS when set (the share
    of the host a job is given), else every core the process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# Floyd-Warshall (Sec. 2, Eq. 1)
# ---------------------------------------------------------------------------

def fw_i32(W: np.ndarray, threads: int = 1) -> np.ndarray:
    """Returns D with D[i][j] = min(shortest i->j distance, INF) (int32)."""
    D = np.array(W, dtype=np.int32, order="C", copy=True)
    n = D.shape[0]
    assert D.shape == (n, n)
    _load().oracle_fw_i32(n, _ptr(D), n, threads)
    return D


def fw_i32_steps(D: np.ndarray, k0: int, k1: int, threads: int = 1) -> np.ndarray:
    """Passes k0 .. k1-1 of the Eq. 1 recurrence applied to a copy of D (int32):
    from W, passes 0 .. k-1 leave the shortest distances whose intermediate
    vertices all lie below k."""
    D = np.array(D, dtype=np.int32, order="C", copy=True)
    n = D.shape[0]
    assert D.shape == (n, n)
    _load().oracle_fw_i32_steps(n, _ptr(D), n, k0, k1, threads)
    return D


def fw_f64(W: np.ndarray, threads: int = 1) -> np.ndarray:
    """fp64 Floyd-Warshall of W promoted to double (+inf = no edge)."""
    D = np.array(W, dtype=np.float64, order="C", copy=True)
    n = D.shape[0]
    assert D.shape == (n, n)
    _load().oracle_fw_f64(n, _ptr(D), n, threads)
    return D


# ---------------------------------------------------------------------------
# Min-plus product (Sec. 3, Eq. 2), accumulating into C
# ---------------------------------------------------------------------------

def minplus_i32(A: np.ndarray, B: np.ndarray, C: np.ndarray | None = None) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    if C is None:
        C = np.full((m, n), INF_I32, dtype=np.int32)
    else:
        C = np.array(C, dtype=np.int32, order="C", copy=True)
    assert C.shape == (m, n)
    _load().oracle_minplus_i32(m, n, k, _ptr(A), max(k, 1), _ptr(B), max(n, 1), _ptr(C), max(n, 1))
    return C


def minplus_f32(A: np.ndarray, B: np.ndarray, C: np.ndarray | None = None) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    if C is None:
        C = np.full((m, n), np.inf, dtype=np.float32)
    else:
        C = np.array(C, dtype=np.float32, order="C", copy=True)
    assert C.shape == (m, n)
    _load().oracle_minplus_f32(m, n, k, _ptr(A), max(k, 1), _ptr(B), max(n, 1), _ptr(C), max(n, 1))
    return C


# ---------------------------------------------------------------------------
# Dijkstra and the Bellman certificate
# ---------------------------------------------------------------------------

def dijkstra_i32(W: np.ndarray, sources, threads: int | None = None) -> np.ndarray:
    """Rows D[s, :] for each source s (int32, clamped to INF)."""
    W = np.ascontiguousarray(W, dtype=np.int32)
    n = W.shape[0]
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    out = np.empty((src.size, n), dtype=np.int32)
    rc = _load().oracle_dijkstra_i32(n, _ptr(W), n, src.size, _ptr(src), _ptr(out),
                                     threads or default_threads())
    if rc != 0:
        raise MemoryError("oracle_dijkstra_i32 failed")
    return out


def dijkstra_f64(W: np.ndarray, sources, threads: int | None = None) -> np.ndarray:
    """Rows D[s, :] in fp64 for fp32 weights W (+inf = no edge)."""
    W = np.ascontiguousarray(W, dtype=np.float32)
    n = W.shape[0]
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    out = np.empty((src.size, n), dtype=np.float64)
    rc = _load().oracle_dijkstra_f64(n, _ptr(W), n, src.size, _ptr(src), _ptr(out),
                                     threads or default_threads())
    if rc != 0:
        raise MemoryError("oracle_dijkstra_f64 failed")
    return out


def certificate_i32(W: np.ndarray, D: np.ndarray, rows=None, threads: int | None = None) -> int:
    """Number of violated Bellman conditions over rows [r0, r1) (0 = D is
    exactly min(APSP(W), INF)).  Requires all finite off-diagonal weights >= 1."""
    W = np.ascontiguousarray(W, dtype=np.int32)
    D = np.ascontiguousarray(D, dtype=np.int32)
    n = W.shape[0]
    r0, r1 = (0, n) if rows is None else rows
    return int(_load().oracle_certificate_i32(n, _ptr(W), n, _ptr(D), n, r0, r1,
                                              threads or default_threads()))


def predecessors_i32(D: np.ndarray, W: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Last-hop predecessor matrix (smallest v != j minimising D[i][v] (+) W[v][j]; -1 when
    i == j or unreachable)."""
    D = np.ascontiguousarray(D, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.int32)
    n = D.shape[0]
    P = np.empty((n, n), dtype=np.int32)
    _load().oracle_predecessors_i32(n, _ptr(D), n, _ptr(W), n, _ptr(P), n, threads or default_threads())
    return P


def walk_weight(W, P, i, j, inf=INF_I32):
    """Follows P back from j to i; returns the path's total cost (None when
    P[i][j] == -1; raises if the walk does not end at i within n steps)."""
    n = len(W)
    if i == j:
        return 0
    if P[i][j] < 0:
        return None
    total, v, steps = 0, j, 0
    while v != i:
        u = int(P[i][v])
        if u < 0 or steps > n:
            raise AssertionError(f"predecessor walk {i}->{j} broken at {v}")
        total += int(W[u][v])
        v = u
        steps += 1
    return total


# ---------------------------------------------------------------------------
# Pure-Python references for tiny inputs
# ---------------------------------------------------------------------------

def brute_apsp(W, inf=INF_I32, saturate=True):
    """Shortest i->j distance by enumerating every simple path (n <= 8).

    With non-negative weights a shortest walk can always be shortened to a
    simple path, so the minimum over simple paths is the APSP value.  For
    int32 (saturate=True) the result is clamped to ``inf``; otherwise a
    missing edge is ``inf`` and sums are exact Python floats/ints."""
    n = len(W)
    assert n <= 8
    out = [[None] * n for _ in range(n)]
    for s in range(n):
        best = [float("inf")] * n
        best[s] = 0

        def dfs(u, dist, seen):
            for v in range(n):
                if v in seen or v == u:
                    continue
                w = W[u][v]
                if (saturate and w >= inf) or (not saturate and w == inf):
                    continue
                nd = dist + w
                if nd < best[v]:
                    best[v] = nd
                dfs(v, nd, seen | {v})

        dfs(s, 0, {s})
        for t in range(n):
            b = best[t]
            if saturate:
                out[s][t] = inf if b >= inf else int(b)
            else:
                out[s][t] = b
    return out


def brute_last_hops(W, inf=INF_I32):
    """For every (i, j) the set of last vertices before j over all shortest
    simple i -> j paths (empty when unreachable or i == j), by enumeration."""
    n = len(W)
    D = brute_apsp(W, inf)
    out = [[set() for _ in range(n)] for _ in range(n)]
    for s in range(n):
        def dfs(u, dist, seen):
            for v in range(n):
                if v in seen or W[u][v] >= inf:
                    continue
                nd = dist + W[u][v]
                if nd == D[s][v] and nd < inf:
                    out[s][v].add(u)
                if nd <= D[s][v]:
                    dfs(v, nd, seen | {v})
        dfs(s, 0, {s})
    return out


def bfs_hops(adj):
    """Hop distances for a boolean adjacency matrix (None = unreachable)."""
    n = len(adj)
    out = []
    for s in range(n):
        dist = [None] * n
        dist[s] = 0
        frontier = [s]
        while frontier:
            nxt = []
            for u in frontier:
                for v in range(n):
                    if adj[u][v] and dist[v] is None:
                        dist[v] = dist[u] + 1
                        nxt.append(v)
            frontier = nxt
        out.append(dist)
    return out


# ---------------------------------------------------------------------------
# Cost-model MLP reference (fp64 numpy): x(4) -> 64 -> 64 -> K, ReLU hidden,
# masked mean-squared error on the targets, Adam.
# ---------------------------------------------------------------------------

def mlp_forward(params, X):
    """Returns (out, cache). params = dict(W1 (4x64), b1, W2 (64x64), b2, W3 (64xK), b3)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ params["W1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ params["W3"] + params["b3"]
    return out, (X, z1, h1, z2, h2)


def mlp_loss(out, T, mask):
    """Masked MSE: sum(mask * (out - T)^2) / max(1, sum(mask))."""
    mask = np.asarray(mask, dtype=np.float64)
    cnt = max(1.0, float(mask.sum()))
    r = (out - T) * mask
    return float((r * r).sum() / cnt)


def mlp_backward(params, cache, out, T, mask):
    """Analytic gradients of mlp_loss with respect to every parameter."""
    X, z1, h1, z2, h2 = cache
    mask = np.asarray(mask, dtype=np.float64)
    cnt = max(1.0, float(mask.sum()))
    g_out = 2.0 * (out - T) * mask / cnt
    g = {}
    g["W3"] = h2.T @ g_out
    g["b3"] = g_out.sum(axis=0)
    g_h2 = g_out @ params["W3"].T
    g_z2 = g_h2 * (z2 > 0)
    g["W2"] = h1.T @ g_z2
    g["b2"] = g_z2.sum(axis=0)
    g_h1 = g_z2 @ params["W2"].T
    g_z1 = g_h1 * (z1 > 0)
    g["W1"] = X.T @ g_z1
    g["b1"] = g_z1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t counts from 1.
    Returns new (params, m, v) without modifying the inputs."""
    newp, newm, newv = {}, {}, {}
    for key in params:
        g = grads[key]
        newm[key] = beta1 * m[key] + (1.0 - beta1) * g
        newv[key] = beta2 * v[key] + (1.0 - beta2) * g * g
        mhat = newm[key] / (1.0 - beta1 ** t)
        vhat = newv[key] / (1.0 - beta2 ** t)
        newp[key] = params[key] - lr * mhat / (np.sqrt(vhat) + eps)
    return newp, newm, newv
