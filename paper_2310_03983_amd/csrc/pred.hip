// Last-hop predecessors (Sec. 2: pred[i][j] is the vertex before j on an
// i -> j path; Sec. 3.1 takes them from an argmin over the intermediate
// index).  Given distances D and costs W:
//
//   P[i][j] = the smallest v != j minimising D[i][v] (+) W[v][j],
//             or -1 when i == j or that minimum is not below INF.
//
// This is one min-plus product D (min,+) W' (W' = W with its diagonal set to
// INF) that also keeps the index of the minimum.  The index forbids the
// packed two-term fold of the distance kernels: every term is an add, a
// compare and two selects.  64 x 64 output tile per workgroup of 256 lanes
// (4 x 4 per lane), reduction staged through LDS in slices of 32; the
// reduction index runs in increasing order with a strict compare, so ties
// keep the smallest v.
#include "device.h"

namespace apsp {

namespace {

constexpr int MT = 64, NT = 64, KT = 32, TM = 4, TN = 4;

template <class S>
__global__ __launch_bounds__(256) void k_predecessors(const typename S::T* __restrict__ D, int64_t ldd,
                                                      const typename S::T* __restrict__ W, int64_t ldw,
                                                      int32_t* __restrict__ P, int64_t ldp, int n,
                                                      const uint32_t* __restrict__ skip_if_set)
{
    using T = typename S::T;
    // the sparse form already wrote P (decided on the device)
    if (skip_if_set && *skip_if_set) return;
    __shared__ T As[KT][MT + 1];   // As[k][row] = D[m0 + row][k0 + k]
    __shared__ T Bs[KT][NT + 1];   // Bs[k][col] = W[k0 + k][n0 + col] (INF on the diagonal)
    const int tiles_n = (n + NT - 1) / NT;
    const int bid = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int m0 = (bid / tiles_n) * MT, n0 = (bid % tiles_n) * NT;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;

    T acc[TM][TN];
    int32_t arg[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            acc[i][j] = S::inf();
            arg[i][j] = -1;
        }

    for (int k0 = 0; k0 < n; k0 += KT) {
        for (int e = tid; e < MT * KT; e += 256) {
            const int row = e / KT, k = e % KT;
            const int gr = m0 + row, gk = k0 + k;
            As[k][row] = (gr < n && gk < n) ? D[(int64_t)gr * ldd + gk] : S::inf();
        }
        for (int e = tid; e < KT * NT; e += 256) {
            const int k = e / NT, col = e % NT;
            const int gk = k0 + k, gc = n0 + col;
            Bs[k][col] = (gk < n && gc < n && gk != gc) ? W[(int64_t)gk * ldw + gc] : S::inf();
        }
        __syncthreads();
        for (int k = 0; k < KT; ++k) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const T s = a[i] + b[j];          // int32: <= 2^31, no wrap
                    if (s < acc[i][j]) {
                        acc[i][j] = s;
                        arg[i][j] = k0 + k;
                    }
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + ty + 16 * i;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int c = n0 + tx + 16 * j;
            if (r < n && c < n) P[(int64_t)r * ldp + c] = (r == c || !(acc[i][j] < S::inf())) ? -1 : arg[i][j];
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse form.  A term D[i][v] (+) W[v][j] can fall below INF only when
// W[v][j] < INF, and v == j is excluded, so P[i][j] is the same argmin taken
// over the in-edges of j alone: n * m candidate terms instead of n^3 for m
// edges.  The columns are cut into ranges of kRange; the edges of each range
// are stored contiguously, ordered by source v, one 64-bit word each:
//   bits 0..15 v, bits 16..31 j - range start, bits 32..63 the cost's bits.
// k_pred_sparse: a workgroup owns kRows rows of D and one column range and
// keeps one 64-bit key per (row, column) in LDS:
//   key = (bits of D[i][v] (+) W[v][j]) << 32 | v,
// folded with an LDS 64-bit atomic min.  Non-negative int32 values and
// non-negative binary32 values both order like their bit patterns, so the
// minimum key is the minimum value, ties broken by the smallest v -- the
// same answer as the dense kernel, whatever order the atomics land in.
// ---------------------------------------------------------------------------
constexpr int kRange = 1024;          // columns per range (j - start fits 16 bits)
constexpr int kRows = 8;              // rows of D per workgroup (LDS keys: 64 KB)

template <class S>
__device__ __forceinline__ bool finite_cost(typename S::T w) { return w < S::inf(); }

// Order-preserving key bits of a non-negative value (fp32: + 0.0f turns a
// -0 sum into +0, which the dense kernel's compare also treats as 0).
__device__ __forceinline__ uint32_t key_bits(uint32_t s) { return s; }
__device__ __forceinline__ uint32_t key_bits(float s) { return __builtin_bit_cast(uint32_t, s + 0.0f); }

// counts[r * n + v] = edges of row v (v -> j, j != v, W finite) with j in range r
template <class S>
__global__ __launch_bounds__(256) void k_edge_count(const typename S::T* __restrict__ W, int64_t ldw, int n,
                                                    int nranges, int32_t* __restrict__ counts)
{
    __shared__ int32_t cnt[64];
    const int v = blockIdx.x;
    for (int r = threadIdx.x; r < nranges; r += 256) cnt[r] = 0;
    __syncthreads();
    const typename S::T* row = W + (int64_t)v * ldw;
    for (int j = threadIdx.x; j < n; j += 256)
        if (j != v && finite_cost<S>(row[j])) atomicAdd(&cnt[j / kRange], 1);
    __syncthreads();
    for (int r = threadIdx.x; r < nranges; r += 256) counts[(int64_t)r * n + v] = cnt[r];
}

// Writes row v's edges of every range at offsets[r * n + v], in increasing j.
template <class S>
__global__ __launch_bounds__(256) void k_edge_fill(const typename S::T* __restrict__ W, int64_t ldw, int n,
                                                   int nranges, const int64_t* __restrict__ offsets,
                                                   uint64_t* __restrict__ edges, const uint32_t* __restrict__ use_sparse)
{
    using T = typename S::T;
    if (!*use_sparse) return;
    __shared__ int32_t wave_tot[4];
    const int v = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const T* row = W + (int64_t)v * ldw;
    for (int r = 0; r < nranges; ++r) {
        int64_t pos = offsets[(int64_t)r * n + v];
        const int j1 = min(n, (r + 1) * kRange);
        for (int c0 = r * kRange; c0 < j1; c0 += 256) {
            const int j = c0 + threadIdx.x;
            T w{};
            bool f = false;
            if (j < j1) {
                w = row[j];
                f = j != v && finite_cost<S>(w);
            }
            const uint64_t mask = __ballot(f);
            const int before = __popcll(mask & ((1ull << lane) - 1ull));
            if (lane == 0) wave_tot[wave] = __popcll(mask);
            __syncthreads();
            int base = 0;
            for (int q = 0; q < wave; ++q) base += wave_tot[q];
            if (f) {
                const uint32_t lo = (uint32_t)v | ((uint32_t)(j - r * kRange) << 16);
                edges[pos + base + before] = ((uint64_t)__builtin_bit_cast(uint32_t, w) << 32) | lo;
            }
            pos += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
            __syncthreads();
        }
    }
}

constexpr int kSparseThreads = 512;   // two workgroups (64 KB of keys each) fill a CU's waves

template <class S>
__global__ __launch_bounds__(kSparseThreads) void k_pred_sparse(const typename S::T* __restrict__ D, int64_t ldd,
                                                                int n, const int64_t* __restrict__ range_start,
                                                                const uint64_t* __restrict__ edges,
                                                                int32_t* __restrict__ P, int64_t ldp,
                                                                const uint32_t* __restrict__ use_sparse)
{
    using T = typename S::T;
    if (!*use_sparse) return;
    __shared__ unsigned long long best[kRows * kRange];
    const int i0 = blockIdx.x * kRows, r = blockIdx.y;
    const int rows = min(kRows, n - i0);
    for (int e = threadIdx.x; e < kRows * kRange; e += kSparseThreads) best[e] = ~0ull;
    __syncthreads();
    const T* Drows = D + (int64_t)i0 * ldd;
    const int64_t e1 = range_start[r + 1];
    // kEdges edges per lane per step: all their D loads are issued before
    // the first atomic, so the loads of one step overlap
    constexpr int kEdges = 4;
    for (int64_t e = range_start[r] + threadIdx.x; e < e1; e += kEdges * kSparseThreads) {
        int v[kEdges], jr[kEdges];
        T w[kEdges], d[kEdges][kRows];
        bool ok[kEdges];
#pragma unroll
        for (int q = 0; q < kEdges; ++q) {
            const int64_t eq = e + (int64_t)q * kSparseThreads;
            ok[q] = eq < e1;
            const uint64_t ed = edges[ok[q] ? eq : e];
            v[q] = (int)(ed & 0xffff);
            jr[q] = (int)((ed >> 16) & 0xffff);
            w[q] = __builtin_bit_cast(T, (uint32_t)(ed >> 32));
        }
#pragma unroll
        for (int q = 0; q < kEdges; ++q)
#pragma unroll
            for (int ii = 0; ii < kRows; ++ii) d[q][ii] = Drows[(int64_t)min(ii, rows - 1) * ldd + v[q]];
#pragma unroll
        for (int ii = 0; ii < kRows; ++ii) {
            if (ii >= rows) break;
#pragma unroll
            for (int q = 0; q < kEdges; ++q) {
                const T sv = d[q][ii] + w[q];   // int32: <= 2^31, no wrap
                if (ok[q])
                    atomicMin(&best[ii * kRange + jr[q]],
                              ((unsigned long long)key_bits(sv) << 32) | (unsigned long long)v[q]);
            }
        }
    }
    __syncthreads();
    const int jbase = r * kRange, width = min(kRange, n - jbase);
    for (int e = threadIdx.x; e < rows * kRange; e += kSparseThreads) {
        const int ii = e / kRange, jr = e - ii * kRange;
        if (jr >= width) continue;
        const int i = i0 + ii, j = jbase + jr;
        const unsigned long long key = best[e];
        const T s = __builtin_bit_cast(T, (uint32_t)(key >> 32));
        const bool none = key == ~0ull || i == j || !(s < S::inf());
        P[(int64_t)i * ldp + j] = none ? -1 : (int32_t)(key & 0xffffffffu);
    }
}


// Edge-list layout on the device: exclusive prefix sums of the range-major
// counts (cells = nranges * n) give offsets[r * n + v]; offsets[cells + r]
// receives the first edge of range r and offsets[cells + nranges] the edge
// total m.  One workgroup: each lane sums a contiguous run of counts, the
// run totals are scanned in LDS, and each lane writes its run's offsets.
// Finally *use_sparse = 1 when the edge list fits (m <= edge_cap) and the
// sparse form is wanted (m <= dense_limit), else 0 (the dense kernel then
// writes P).
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_edge_scan(const int32_t* __restrict__ counts, int64_t cells,
                                                            int32_t n, int nranges, int64_t* __restrict__ offsets,
                                                            int64_t edge_cap, int64_t dense_limit,
                                                            uint32_t* __restrict__ use_sparse)
{
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (cells + kScanThreads - 1) / kScanThreads;
    const int64_t b = min(cells, (int64_t)t * per), e = min(cells, b + per);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // inclusive scan of the run totals
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    // range starts are the offsets at indices r * n
    int64_t r = (b + n - 1) / n, boundary = r * n;
    for (int64_t i = b; i < e; ++i) {
        if (i == boundary) {
            offsets[cells + r] = run;
            ++r;
            boundary += n;
        }
        offsets[i] = run;
        run += counts[i];
    }
    if (t == kScanThreads - 1) {
        const int64_t m = part[kScanThreads - 1];
        offsets[cells + nranges] = m;
        *use_sparse = (m <= edge_cap && m <= dense_limit) ? 1u : 0u;
    }
}

// Path reconstruction (Sec. 2: the path is recovered by following the
// predecessor of the target back to the source).  One lane per query: the
// first walk counts the vertices, the second writes them source first.  A
// predecessor outside [0, n), a chain longer than max_len vertices (or than
// n) gives length -1; an unreachable target (P[s][t] < 0, s != t) gives 0.
__global__ __launch_bounds__(256) void k_paths(const int32_t* __restrict__ P, int64_t ldp, int32_t n, int32_t count,
                                               const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                               int32_t* __restrict__ paths, int32_t max_len,
                                               int32_t* __restrict__ len)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int32_t s = src[q], t = dst[q];
    int32_t* out = paths + (int64_t)q * max_len;
    if (s < 0 || s >= n || t < 0 || t >= n) {
        len[q] = -1;
        return;
    }
    const int32_t* row = P + (int64_t)s * ldp;
    if (s != t && row[t] < 0) {
        len[q] = 0;
        return;
    }
    const int32_t limit = min(max_len, n);
    int32_t L = 1, v = t;
    while (v != s) {
        const int32_t u = row[v];
        if (u < 0 || u >= n || L >= limit) {
            len[q] = -1;
            return;
        }
        v = u;
        ++L;
    }
    v = t;
    for (int32_t i = L - 1; i >= 0; --i) {
        out[i] = v;
        if (i) v = row[v];
    }
    len[q] = L;
}

}  // namespace

int pred_sparse_ranges(int32_t n) { return (n + kRange - 1) / kRange; }

hipError_t launch_edge_count(DType dt, const void* W, int64_t ldw, int32_t n, int32_t* counts, hipStream_t st)
{
    const int nr = pred_sparse_ranges(n);
    if (dt == I32)
        hipLaunchKernelGGL(k_edge_count<dev::SemI32>, dim3(n), dim3(256), 0, st, (const uint32_t*)W, ldw, n, nr,
                           counts);
    else
        hipLaunchKernelGGL(k_edge_count<dev::SemF32>, dim3(n), dim3(256), 0, st, (const float*)W, ldw, n, nr,
                           counts);
    return hipGetLastError();
}

hipError_t launch_edge_scan(const int32_t* counts, int32_t n, int64_t* offsets, int64_t edge_cap,
                            int64_t dense_limit, uint32_t* use_sparse, hipStream_t st)
{
    const int nr = pred_sparse_ranges(n);
    hipLaunchKernelGGL(k_edge_scan, dim3(1), dim3(kScanThreads), 0, st, counts, (int64_t)nr * n, n, nr, offsets,
                       edge_cap, dense_limit, use_sparse);
    return hipGetLastError();
}

hipError_t launch_pred_sparse(DType dt, const void* D, int64_t ldd, const void* W, int64_t ldw, int32_t* P,
                              int64_t ldp, int32_t n, const int64_t* offsets, const int64_t* range_start,
                              uint64_t* edges, const uint32_t* use_sparse, hipStream_t st)
{
    const int nr = pred_sparse_ranges(n);
    const dim3 grid((unsigned)((n + kRows - 1) / kRows), (unsigned)nr);
    if (dt == I32) {
        hipLaunchKernelGGL(k_edge_fill<dev::SemI32>, dim3(n), dim3(256), 0, st, (const uint32_t*)W, ldw, n, nr,
                           offsets, edges, use_sparse);
        hipLaunchKernelGGL(k_pred_sparse<dev::SemI32>, grid, dim3(kSparseThreads), 0, st, (const uint32_t*)D, ldd,
                           n, range_start, edges, P, ldp, use_sparse);
    } else {
        hipLaunchKernelGGL(k_edge_fill<dev::SemF32>, dim3(n), dim3(256), 0, st, (const float*)W, ldw, n, nr,
                           offsets, edges, use_sparse);
        hipLaunchKernelGGL(k_pred_sparse<dev::SemF32>, grid, dim3(kSparseThreads), 0, st, (const float*)D, ldd,
                           n, range_start, edges, P, ldp, use_sparse);
    }
    return hipGetLastError();
}

hipError_t launch_paths(const int32_t* P, int64_t ldp, int32_t n, int32_t count, const int32_t* src,
                        const int32_t* dst, int32_t* paths, int32_t max_len, int32_t* len, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_paths, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, P, ldp, n, count, src, dst,
                       paths, max_len, len);
    return hipGetLastError();
}

hipError_t launch_predecessors(DType dt, const void* D, int64_t ldd, const void* W, int64_t ldw, int32_t* P,
                               int64_t ldp, int32_t n, const uint32_t* skip_if_set, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (int64_t)((n + MT - 1) / MT) * ((n + NT - 1) / NT);
    if (dt == I32)
        hipLaunchKernelGGL(k_predecessors<dev::SemI32>, dim3((unsigned)tiles), dim3(256), 0, st,
                           (const uint32_t*)D, ldd, (const uint32_t*)W, ldw, P, ldp, n, skip_if_set);
    else
        hipLaunchKernelGGL(k_predecessors<dev::SemF32>, dim3((unsigned)tiles), dim3(256), 0, st,
                           (const float*)D, ldd, (const float*)W, ldw, P, ldp, n, skip_if_set);
    return hipGetLastError();
}

}  // namespace apsp
