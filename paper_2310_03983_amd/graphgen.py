"""Seeded synthetic graph generator (shared by the tests, the benchmark and the
oracle checks; it contains no APSP arithmetic).

Shape of the generator follows the paper's Sec. 3.4: an independent Bernoulli
draw decides each directed edge, each present edge gets a uniformly drawn
cost, the diagonal is 0.  Absent edges get INF (int32: 2**30; fp32: +inf).

Every random number is counter-based, so any entry can be regenerated on its
own and the output does not depend on chunking or thread count:

    mix64(z)   = SplitMix64 finalizer (Steele, Lea & Flood, OOPSLA 2014)
    h(s, t, x) = mix64(mix64(s + t * 0x9E3779B97F4A7C15) + x)     (mod 2**64)
    u01(h)     = (h >> 11) * 2**-53

with stream ids t: EDGE=1, WEIGHT=2, N=3, P=4, PERM=5, SRC=6, CHAIN=7 and
x = i * n + j for per-entry streams.  The seed of graph g of a workload with
base seed S is mix64(S + g).
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import os
from dataclasses import dataclass

import numpy as np

INF_I32 = 1 << 30
GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1

EDGE, WEIGHT, NSTREAM, PSTREAM, PERM, SRC, CHAIN = 1, 2, 3, 4, 5, 6, 7
COUNTSTREAM, HISTREAM, LOSTREAM = 8, 9, 10   # batch sweep: graph count, largest n, smallest n


# --------------------------------------------------------------------------
# counter-based hashing
# --------------------------------------------------------------------------

def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, stream: int) -> int:
    return mix64((seed + stream * GOLDEN) & M64)


def h(seed: int, stream: int, x: int) -> int:
    return mix64((stream_key(seed, stream) + x) & M64)


def h_np(seed: int, stream: int, x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        return mix64_np(np.uint64(stream_key(seed, stream)) + x.astype(np.uint64))


def u01(v: int) -> float:
    return (v >> 11) * (2.0 ** -53)


def u01_np(v: np.ndarray) -> np.ndarray:
    return (v >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def graph_seed(base_seed: int, g: int) -> int:
    return mix64(base_seed + g)


def _uniform_int_np(hv: np.ndarray, lo: int, hi: int) -> np.ndarray:
    span = np.uint64(hi - lo + 1)
    with np.errstate(over="ignore"):
        return (np.int64(lo) + ((hv >> np.uint64(32)) * span >> np.uint64(32)).astype(np.int64))


def _uniform_int(hv: int, lo: int, hi: int) -> int:
    return lo + (((hv >> 32) * (hi - lo + 1)) >> 32)


# --------------------------------------------------------------------------
# single graphs
# --------------------------------------------------------------------------

def _edge_mask_rows(seed: int, n: int, p: float, r0: int, r1: int) -> np.ndarray:
    i = np.arange(r0, r1, dtype=np.uint64)[:, None]
    j = np.arange(n, dtype=np.uint64)[None, :]
    x = i * np.uint64(n) + j
    mask = u01_np(h_np(seed, EDGE, x)) < p
    idx = np.arange(r0, r1)
    mask[idx - r0, idx] = False
    return mask


def _for_chunks(fn, n, chunk_rows):
    """Runs fn(r0) for every row chunk; chunks write disjoint rows and every
    value is counter-based, so threads do not change the output."""
    starts = list(range(0, n, chunk_rows))
    workers = min(len(starts), max(1, min(os.cpu_count() or 1, 8)))
    if workers <= 1:
        for r0 in starts:
            fn(r0)
        return
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fn, starts))


def graph_i32(n: int, p: float, lo: int, hi: int, seed: int, chunk_rows: int = 1024) -> np.ndarray:
    """Directed graph, edge i->j (i != j) with probability p, integer cost
    uniform in [lo, hi]; diagonal 0, absent edges INF = 2**30."""
    assert 0 <= lo <= hi < INF_I32
    W = np.full((n, n), INF_I32, dtype=np.int32)

    def rows(r0):
        r1 = min(n, r0 + chunk_rows)
        mask = _edge_mask_rows(seed, n, p, r0, r1)
        ii, jj = np.nonzero(mask)
        x = (ii.astype(np.uint64) + np.uint64(r0)) * np.uint64(n) + jj.astype(np.uint64)
        W[ii + r0, jj] = _uniform_int_np(h_np(seed, WEIGHT, x), lo, hi).astype(np.int32)

    _for_chunks(rows, n, chunk_rows)
    np.fill_diagonal(W, 0)
    return W


def graph_f32(n: int, p: float, lo: float, hi: float, seed: int, chunk_rows: int = 1024) -> np.ndarray:
    """Same topology stream as graph_i32; cost = float32(lo + (hi-lo)*u),
    u in [0,1) computed in double and rounded once; absent edges +inf."""
    W = np.full((n, n), np.inf, dtype=np.float32)

    def rows(r0):
        r1 = min(n, r0 + chunk_rows)
        mask = _edge_mask_rows(seed, n, p, r0, r1)
        ii, jj = np.nonzero(mask)
        x = (ii.astype(np.uint64) + np.uint64(r0)) * np.uint64(n) + jj.astype(np.uint64)
        w = lo + (hi - lo) * u01_np(h_np(seed, WEIGHT, x))
        W[ii + r0, jj] = w.astype(np.float32)

    _for_chunks(rows, n, chunk_rows)
    np.fill_diagonal(W, 0.0)
    return W


def permutation(seed: int, n: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by the PERM stream."""
    perm = list(range(n))
    key = stream_key(seed, PERM)
    for t in range(n - 1, 0, -1):
        j = _uniform_int(mix64((key + t) & M64), 0, t)
        perm[t], perm[j] = perm[j], perm[t]
    return np.asarray(perm, dtype=np.int64)


def add_chain_i32(W: np.ndarray, seed: int, lo: int, hi: int) -> np.ndarray:
    """Adds edges perm[t] -> perm[t+1] (weight from the CHAIN stream) where no
    Bernoulli edge exists, which makes the graph weakly connected."""
    n = W.shape[0]
    perm = permutation(seed, n)
    key = stream_key(seed, CHAIN)
    for t in range(n - 1):
        a, b = int(perm[t]), int(perm[t + 1])
        if W[a, b] >= INF_I32:
            W[a, b] = _uniform_int(mix64((key + t) & M64), lo, hi)
    return W


def dijkstra_sources(n: int, seed: int, count: int = 64) -> np.ndarray:
    """{0, n-1} then the first distinct h(seed, SRC, t) mod n; all vertices
    when n <= count."""
    if n <= count:
        return np.arange(n, dtype=np.int64)
    out = [0, n - 1]
    seen = set(out)
    t = 0
    while len(out) < count:
        v = h(seed, SRC, t) % n
        t += 1
        if v not in seen:
            seen.add(v)
            out.append(v)
    return np.asarray(out, dtype=np.int64)


def log_uniform_int(seed: int, stream: int, a: int, b: int) -> int:
    u = u01(h(seed, stream, 0))
    v = int(round(math.exp(math.log(a) + u * (math.log(b) - math.log(a)))))
    return min(max(v, a), b)


def log_uniform(seed: int, stream: int, a: float, b: float) -> float:
    u = u01(h(seed, stream, 0))
    return math.exp(math.log(a) + u * (math.log(b) - math.log(a)))


def uniform(seed: int, stream: int, a: float, b: float) -> float:
    return a + (b - a) * u01(h(seed, stream, 0))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Single:
    """One directed graph: n vertices, edge probability p, cost range."""
    name: str
    n: int
    p: float
    dtype: str          # "i32" | "f32"
    lo: float
    hi: float
    base_seed: int

    def seed(self) -> int:
        return graph_seed(self.base_seed, 0)

    def make(self) -> np.ndarray:
        if self.dtype == "i32":
            return graph_i32(self.n, self.p, int(self.lo), int(self.hi), self.seed())
        return graph_f32(self.n, self.p, self.lo, self.hi, self.seed())

    def sources(self, count: int = 64) -> np.ndarray:
        return dijkstra_sources(self.n, self.seed(), count)


SINGLE = {
    "n256_p0.1_i32": Single("n256_p0.1_i32", 256, 0.1, "i32", 1, 100, 1),
    "n4096_p0.05_i32": Single("n4096_p0.05_i32", 4096, 0.05, "i32", 1, 1000, 2),
    "n16384_p0.01_f32": Single("n16384_p0.01_f32", 16384, 0.01, "f32", 0.1, 10.0, 3),
    # int32 companion of the n=16384 graph: same topology seed, C-range weights
    "n16384_p0.01_i32": Single("n16384_p0.01_i32", 16384, 0.01, "i32", 1, 1000, 3),
}


@dataclass(frozen=True)
class BatchGraph:
    g: int
    n: int
    p: float
    seed: int


def batch_ragged(count: int = 512, n_lo: int = 32, n_hi: int = 512,
                 p_lo: float = 0.02, p_hi: float = 0.3, base_seed: int = 4):
    """Independent graphs, n log-uniform in [n_lo, n_hi], p uniform in
    [p_lo, p_hi] (the 512-graph batched workload)."""
    out = []
    for g in range(count):
        s = graph_seed(base_seed, g)
        n = log_uniform_int(s, NSTREAM, n_lo, n_hi)
        p = uniform(s, PSTREAM, p_lo, p_hi)
        out.append(BatchGraph(g, n, p, s))
    return out


def batch_graph_i32(bg: BatchGraph, lo: int = 1, hi: int = 100) -> np.ndarray:
    return graph_i32(bg.n, bg.p, lo, hi, bg.seed)


@dataclass(frozen=True)
class SweepGraph:
    g: int
    n: int
    p: float
    chain: bool
    seed: int


def sweep(count: int = 200, n_lo: int = 64, n_hi: int = 32768,
          p_lo: float = 5e-4, p_hi: float = 0.5, base_seed: int = 5):
    """The cost-model sweep: n and p log-uniform; even g get a seeded spanning
    chain (weakly connected), odd g are Bernoulli only."""
    out = []
    for g in range(count):
        s = graph_seed(base_seed, g)
        n = log_uniform_int(s, NSTREAM, n_lo, n_hi)
        p = log_uniform(s, PSTREAM, p_lo, p_hi)
        out.append(SweepGraph(g, n, p, g % 2 == 0, s))
    return out


def sweep_graph_i32(sg: SweepGraph, lo: int = 1, hi: int = 1000) -> np.ndarray:
    W = graph_i32(sg.n, sg.p, lo, hi, sg.seed)
    if sg.chain:
        add_chain_i32(W, sg.seed, lo, hi)
    return W


@dataclass(frozen=True)
class BatchSpec:
    """One batch of the batch sweep: `count` graphs with n log-uniform in
    [n_lo, n_hi] and p uniform in [p_lo, p_hi], drawn like the 512-graph
    workload with its own base seed."""
    b: int
    count: int
    n_lo: int
    n_hi: int
    p_lo: float
    p_hi: float
    base_seed: int

    def graphs(self):
        return batch_ragged(self.count, self.n_lo, self.n_hi, self.p_lo, self.p_hi, self.base_seed)


def batch_sweep(count: int = 200, base_seed: int = 6):
    """Batches for timing the batched schedules (the batch cost model's
    data).  Batches 0..159: graph count log-uniform in [16, 768], largest n
    log-uniform in [96, 1024], smallest n 32 or 64, p uniform in
    [0.02, p_hi] with p_hi uniform in [0.05, 0.3].  Batches 160..199 cover
    large dense batches more closely: count log-uniform in [256, 768],
    smallest n 32, largest n log-uniform in [384, 640], p_hi uniform in
    [0.2, 0.3].  Costs 1..100 as in the 512-graph workload."""
    out = []
    for b in range(count):
        s = graph_seed(base_seed, b)
        if b < 160:
            cnt = log_uniform_int(s, COUNTSTREAM, 16, 768)
            n_hi = log_uniform_int(s, HISTREAM, 96, 1024)
            n_lo = 32 if u01(h(s, LOSTREAM, 0)) < 0.5 else 64
            p_hi = uniform(s, PSTREAM, 0.05, 0.3)
        else:
            cnt = log_uniform_int(s, COUNTSTREAM, 256, 768)
            n_hi = log_uniform_int(s, HISTREAM, 384, 640)
            n_lo = 32
            p_hi = uniform(s, PSTREAM, 0.2, 0.3)
        out.append(BatchSpec(b, cnt, n_lo, n_hi, 0.02, p_hi, 1000 + b))
    return out


def pack_batch(mats):
    """Concatenates row-major square matrices; returns (flat, offsets, sizes)
    with offsets in elements."""
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    counts = sizes.astype(np.int64) ** 2
    offsets = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        offsets[1:] = np.cumsum(counts)[:-1]
    flat = np.concatenate([m.ravel() for m in mats]) if mats else np.zeros(0, np.int32)
    return flat, offsets, sizes
