// Planner features of one graph, computed on the device from its cost
// matrix: the edge count m (finite off-diagonal entries; density =
// m / (n (n - 1)), the generator's directed density, Sec. 3.4) and whether
// the graph is weakly connected (edges taken as undirected).
//
// One pass over the matrix counts the edges and joins the two ends of every
// edge in a union-find forest held in the workspace (one int32 parent per
// vertex).  The forest is lock-free: a root is hooked only under a smaller
// root, by a compare-and-swap that succeeds only while it is still a root,
// so parent[x] <= x always holds, every chain strictly decreases and every
// walk ends; a failed swap returns the root's new parent, from which the
// walk resumes.  Finds halve the path by swapping a vertex's parent for its
// grandparent (again only by compare-and-swap), and the far end of a joined
// edge is pointed straight at the root the join ended with, so that the
// common case -- an edge inside the tree, whose far end hangs right below the
// root -- costs one cached read.  A second pass (one workgroup) counts the
// roots: the graph is weakly connected iff there is exactly one.  Graphs
// below 1024 vertices take one workgroup instead, with the forest in LDS.
#include "device.h"
#include "internal.h"

#include <algorithm>
#include <type_traits>

namespace apsp {

namespace {

constexpr int kThreads = 256;
constexpr int32_t kSampleMinN = 1024;   // graphs from this size take the sampled passes, smaller ones one workgroup

// Parent reads go through the caches and may return an older parent: every
// value a vertex ever had is an ancestor of it (parents only move up), so a
// walk still ends at a vertex of the same tree, and any link is changed only
// by a compare-and-swap, which sees the current value.
__device__ __forceinline__ int32_t load_parent(int32_t* parent, int32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x)
{
    int32_t p = load_parent(parent, x);
    while (p != x) {
        const int32_t g = load_parent(parent, p);
        if (g != p) atomicCAS(parent + x, p, g);   // path halving; a no-op if x moved meanwhile
        x = p;
        p = g;
    }
    return x;
}

// Joins the tree of j (a neighbour of the row's vertex) with the row's tree,
// whose root was ri, and leaves in ri a root the two trees then had; j is
// then pointed straight at that root, so later edges to j take the fast test.
__device__ __forceinline__ void join(int32_t* parent, int32_t& ri, int32_t j)
{
    int32_t a = find_root(parent, ri), b = find_root(parent, j);
    while (a != b) {
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // hook the larger root b under a, if b is still a root
        const int32_t old = atomicCAS(parent + b, b, a);
        if (old == b) break;
        b = find_root(parent, old);   // b was hooked meanwhile: continue from its new root
        a = find_root(parent, a);
    }
    ri = a;
    // a is an ancestor of j and not above j's current parent only if the
    // parent is already a or higher; otherwise move j up to a
    const int32_t pj = load_parent(parent, j);
    if (pj > a) atomicCAS(parent + j, pj, a);
}

template <class T>
__device__ __forceinline__ bool edge(T w);
template <>
__device__ __forceinline__ bool edge<uint32_t>(uint32_t w) { return w < kInfI32; }
template <>
__device__ __forceinline__ bool edge<float>(float w) { return w < __builtin_inff(); }

// Zeroes the two counters and makes every vertex its own root.
__global__ __launch_bounds__(kThreads) void k_features_init(int32_t* parent, int32_t n, unsigned long long* edges,
                                                            uint32_t* roots)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *edges = 0ull;
        *roots = 0u;
    }
    for (int32_t v = blockIdx.x * kThreads + threadIdx.x; v < n; v += gridDim.x * kThreads) parent[v] = v;
}

// Rows are taken by workgroups and read four elements per access, four
// accesses in flight per lane.  Each lane keeps a root of the row's tree; an
// edge whose other end has that vertex as its parent is already inside the
// tree and skips the join.
//
// Passes: kSample counts every edge and records at most
// kWaveSample of them per wave and row (the lowest marked column of the
// first lanes, in lane order, that have one) in LDS; the workgroup joins the
// recorded edges after its last row, one lane per row and wave, so that the
// latency of the joins does not hold up the stream of loads.  If the
// sampled subgraph is already connected, so is the graph, and kRest (which
// joins every edge, without counting) returns at once; otherwise kRest
// completes the forest.  On a Bernoulli graph a few edges per vertex
// connect it, so the common case joins a small fraction of the edges.
//
// The count is branch-free: a lane folds the finite tests of its sixteen
// elements into one mask and adds its population count; only lanes with a
// marked element enter the join or record code.
enum JoinPass { kSample = 1, kRest = 2 };
constexpr int kWaveSample = 4;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxSampleRows = 64;   // rows of one workgroup in the sampled pass (the launch ensures it)

// Joins every edge marked in mask (bit b: column col0 + (b / 4) * stride +
// b % 4) to the row's tree.
__device__ __forceinline__ void join_marked(int32_t* parent, int32_t& ri, uint32_t mask, int32_t col0, int32_t stride)
{
    while (mask) {
        const int b = __builtin_ctz(mask);
        mask &= mask - 1u;
        const int32_t c = col0 + (b >> 2) * stride + (b & 3);
        if (load_parent(parent, c) != ri) join(parent, ri, c);
    }
}

// Records the lowest marked column of this lane in the wave's next free
// slot of the row, for the first kWaveSample marked lanes; taken counts the
// wave's marked lanes so far in the row.  (Where lanes have diverged, two
// may pick one slot or leave one empty: a slot only ever holds -1 or an
// edge of the row.)
__device__ __forceinline__ void sample_marked(int32_t* slots, uint32_t mask, int32_t col0, int32_t stride, int& taken)
{
    if (taken >= kWaveSample) return;
    const unsigned long long voters = __ballot(mask != 0u);
    if (mask) {
        const int lane = threadIdx.x & 63;
        const int slot = taken + __popcll(voters & ((1ull << lane) - 1ull));
        if (slot < kWaveSample) {
            const int b = __builtin_ctz(mask);
            slots[slot] = col0 + (b >> 2) * stride + (b & 3);
        }
    }
    taken += __popcll(voters);
}

// Bit e of the result: element e of the four (columns c .. c + 3) is an edge.
template <class T>
__device__ __forceinline__ uint32_t edge_bits(const dev::Pair2<dev::Pair2<T>>& v, int32_t c, int32_t r)
{
    return (uint32_t)(edge<T>(v.x.x) && c != r) | ((uint32_t)(edge<T>(v.x.y) && c + 1 != r) << 1) |
           ((uint32_t)(edge<T>(v.y.x) && c + 2 != r) << 2) | ((uint32_t)(edge<T>(v.y.y) && c + 3 != r) << 3);
}

template <class T, int PASS>
__global__ __launch_bounds__(kThreads) void k_graph_edges(const T* __restrict__ D, int32_t n, int64_t ld,
                                                          int32_t* parent, unsigned long long* edges,
                                                          const uint32_t* connected)
{
    using V = dev::Pair2<dev::Pair2<T>>;   // four elements, one dwordx4 access
    constexpr int kStep = 4 * kThreads;
    if constexpr (PASS == kRest) {
        if (*connected) return;   // the sample already connected the graph
    }
    constexpr int kSlots = PASS == kSample ? kMaxSampleRows * kWaves * kWaveSample : 1;
    __shared__ int32_t s_slots[kSlots];   // recorded edges, by (local row, wave, slot); -1 = none
    if constexpr (PASS == kSample) {
        for (int i = threadIdx.x; i < kSlots; i += kThreads) s_slots[i] = -1;
        __syncthreads();
    }
    uint32_t cnt = 0;
    int rows = 0;   // rows this workgroup has taken
    for (int32_t r = blockIdx.x; r < n; r += gridDim.x, ++rows) {
        const T* row = D + (int64_t)r * ld;
        int32_t ri = r;
        if constexpr (PASS != kSample) ri = find_root(parent, r);
        // kSample: this wave's slots of the row; past kMaxSampleRows rows
        // nothing is recorded (taken starts full)
        const bool record = PASS == kSample && rows < kMaxSampleRows;
        int32_t* slots = nullptr;
        if constexpr (PASS == kSample)
            slots = s_slots + ((record ? rows : 0) * kWaves + (threadIdx.x >> 6)) * kWaveSample;
        int taken = record ? 0 : kWaveSample;
        auto visit = [&](uint32_t mask, int32_t col0, int32_t stride) {
            if constexpr (PASS != kRest) cnt += __popc(mask);
            if constexpr (PASS == kSample) sample_marked(slots, mask, col0, stride, taken);
            else join_marked(parent, ri, mask, col0, stride);
        };
        int32_t c = threadIdx.x * 4;
        for (; c + 3 * kStep + 3 < n; c += 4 * kStep) {
            V v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = dev::ld_vec<V>(row + c + q * kStep);
            uint32_t mask = 0;   // bit 4q + e: element e of access q
#pragma unroll
            for (int q = 0; q < 4; ++q) mask |= edge_bits<T>(v[q], c + q * kStep, r) << (4 * q);
            visit(mask, c, kStep);
        }
        for (; c + 3 < n; c += kStep) visit(edge_bits<T>(dev::ld_vec<V>(row + c), c, r), c, kStep);
        for (; c < n; ++c) visit((edge<T>(row[c]) && c != r) ? 1u : 0u, c, 0);
    }
    if constexpr (PASS == kSample) {
        // the recorded edges: one lane per (row, wave), its slots in order
        __syncthreads();
        const int pairs = (rows < kMaxSampleRows ? rows : kMaxSampleRows) * kWaves;
        for (int i = threadIdx.x; i < pairs; i += kThreads) {
            const int32_t r = blockIdx.x + (i / kWaves) * gridDim.x;
            int32_t ri = find_root(parent, r);
            for (int k = 0; k < kWaveSample; ++k) {
                const int32_t c = s_slots[i * kWaveSample + k];
                if (c < 0) break;
                if (load_parent(parent, c) != ri) join(parent, ri, c);
            }
        }
    }
    if constexpr (PASS != kRest) {
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        __shared__ uint32_t part[kThreads / 64];
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < kThreads / 64; ++w) tot += part[w];
            if (tot) atomicAdd(edges, tot);
        }
    }
}

// One workgroup: *connected = 1 when the forest has one root.
constexpr int kRootThreads = 1024;
__global__ __launch_bounds__(kRootThreads) void k_one_root(const int32_t* parent, int32_t n, uint32_t* connected)
{
    uint32_t cnt = 0;
    for (int32_t v = threadIdx.x; v < n; v += kRootThreads) cnt += parent[v] == v;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    __shared__ uint32_t part[kRootThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t roots = 0;
        for (int w = 0; w < kRootThreads / 64; ++w) roots += part[w];
        *connected = roots == 1u ? 1u : 0u;
    }
}

// The cost model's inputs of one graph: log2 n, log10 density (clamped to
// 1e-9), log2 batch, weakly connected (1 / 0; a graph of one vertex or none
// is connected).
__device__ void write_features(float* x, int32_t n, int32_t batch, unsigned long long edges, bool connected)
{
    const double pairs = (double)n * (double)(n > 1 ? n - 1 : 1);
    const double dens = fmax((double)edges / pairs, 1e-9);
    x[0] = (float)log2((double)(n > 1 ? n : 1));
    x[1] = (float)log10(dens);
    x[2] = (float)log2((double)(batch > 1 ? batch : 1));
    x[3] = (n <= 1 || connected) ? 1.f : 0.f;
}

// One workgroup: counts the roots of the forest, then writes the cost
// model's inputs: log2 n, log10 density (clamped to 1e-9), log2 batch,
// weakly connected (1 / 0; a graph of one vertex or none is connected).
constexpr int kFinishThreads = 1024;
__global__ __launch_bounds__(kFinishThreads) void k_features_finish(const int32_t* parent, int32_t n, int32_t batch,
                                                                    const unsigned long long* edges, float* x)
{
    uint32_t cnt = 0;
    for (int32_t v = threadIdx.x; v < n; v += kFinishThreads) cnt += parent[v] == v;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    __shared__ uint32_t part[kFinishThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t roots = 0;
    for (int w = 0; w < kFinishThreads / 64; ++w) roots += part[w];
    write_features(x, n, batch, *edges, roots == 1u);
}

// Graphs below kSampleMinN vertices: one workgroup computes the features in
// one launch, with the union-find forest in LDS (the same forest and rules
// as above; LDS atomics cost a fraction of device-scope ones).  Waves take
// kSmallRows rows at a time, one 16-byte access per row in flight per lane,
// and join every edge; then the roots are counted.  (One workgroup reads
// about 25 GB/s here: at n = 256 it takes 19 us against 58 for the
// multi-workgroup passes, at n = 1024 166 against 98.)
constexpr int32_t kSmallMaxN = kSampleMinN - 1;
constexpr int kSmallThreads = 1024;
constexpr int kSmallRows = 8;

__device__ __forceinline__ int32_t lds_parent(int32_t* par, int32_t x)
{
    return __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ int32_t lds_find(int32_t* par, int32_t x)
{
    int32_t p = lds_parent(par, x);
    while (p != x) {
        const int32_t g = lds_parent(par, p);
        if (g != p) atomicCAS(par + x, p, g);
        x = p;
        p = g;
    }
    return x;
}

__device__ void lds_join(int32_t* par, int32_t a, int32_t b)
{
    a = lds_find(par, a);
    b = lds_find(par, b);
    while (a != b) {
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(par + b, b, a);   // hook root b under the smaller root a
        if (old == b) return;
        b = lds_find(par, old);
        a = lds_find(par, a);
    }
}

template <class T>
__global__ __launch_bounds__(kSmallThreads) void k_features_small(const T* __restrict__ D, int32_t n, int64_t ld,
                                                                  unsigned long long* edges, float* x)
{
    using V = dev::Pair2<dev::Pair2<T>>;
    constexpr int kW = kSmallThreads / 64;
    __shared__ int32_t par[kSmallMaxN + 1];
    __shared__ uint32_t s_cnt[kW], s_roots[kW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int32_t v = tid; v < n; v += kSmallThreads) par[v] = v;
    __syncthreads();
    uint32_t cnt = 0;
    for (int32_t r0 = wave * kSmallRows; r0 < n; r0 += kW * kSmallRows) {
        const int rows = n - r0 < kSmallRows ? n - r0 : kSmallRows;
        for (int32_t c = lane * 4; c < n; c += 256) {
            if (c + 3 < n) {
                V v[kSmallRows];
#pragma unroll
                for (int q = 0; q < kSmallRows; ++q)
                    if (q < rows) v[q] = dev::ld_vec<V>(D + (int64_t)(r0 + q) * ld + c);
#pragma unroll
                for (int q = 0; q < kSmallRows; ++q) {
                    if (q >= rows) break;
                    uint32_t m = edge_bits<T>(v[q], c, r0 + q);
                    cnt += __popc(m);
                    while (m) {
                        const int b = __builtin_ctz(m);
                        m &= m - 1u;
                        lds_join(par, r0 + q, c + b);
                    }
                }
            } else {
                for (int q = 0; q < rows; ++q)
                    for (int32_t cc = c; cc < n; ++cc)
                        if (cc != r0 + q && edge<T>(D[(int64_t)(r0 + q) * ld + cc])) {
                            ++cnt;
                            lds_join(par, r0 + q, cc);
                        }
            }
        }
    }
    __syncthreads();
    uint32_t roots = 0;
    for (int32_t v = tid; v < n; v += kSmallThreads) roots += lds_parent(par, v) == v;
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off);
        roots += __shfl_xor(roots, off);
    }
    if (lane == 0) {
        s_cnt[wave] = cnt;
        s_roots[wave] = roots;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long tot = 0;
        uint32_t rt = 0;
        for (int w = 0; w < kW; ++w) {
            tot += s_cnt[w];
            rt += s_roots[w];
        }
        *edges = tot;
        write_features(x, n, 1, tot, rt == 1u);
    }
}

}  // namespace

hipError_t launch_graph_features(DType dt, const void* D, int32_t n, int64_t ld, int32_t* parent,
                                 unsigned long long* edges, uint32_t* roots, float* x, hipStream_t st)
{
    if (n <= kSmallMaxN) {
        if (dt == F32)
            hipLaunchKernelGGL(k_features_small<float>, dim3(1), dim3(kSmallThreads), 0, st,
                               static_cast<const float*>(D), n > 1 ? n : 0, ld, edges, x);
        else
            hipLaunchKernelGGL(k_features_small<uint32_t>, dim3(1), dim3(kSmallThreads), 0, st,
                               static_cast<const uint32_t*>(D), n > 1 ? n : 0, ld, edges, x);
        return hipGetLastError();
    }
    const int gi = (int)std::min<int64_t>(std::max<int64_t>((n + kThreads - 1) / kThreads, 1), 1024);
    hipLaunchKernelGGL(k_features_init, dim3(gi), dim3(kThreads), 0, st, parent, n > 1 ? n : 0, edges, roots);
    if (n > 1) {
        // at most kMaxSampleRows rows per workgroup
        const int gr = (int)std::max<int64_t>(std::min<int64_t>(n, 4096), (n + kMaxSampleRows - 1) / kMaxSampleRows);
        auto pass = [&](auto tag, auto pass_c) {
            using T = decltype(tag);
            constexpr int PASS = decltype(pass_c)::value;
            hipLaunchKernelGGL((k_graph_edges<T, PASS>), dim3(gr), dim3(kThreads), 0, st, static_cast<const T*>(D), n,
                               ld, parent, edges, roots);
        };
        using Sample = std::integral_constant<int, kSample>;
        using Rest = std::integral_constant<int, kRest>;
        // sampled joins, the one-root test (roots is its flag word), then
        // the remaining joins unless the sample connected the graph
        if (dt == F32) pass(float{}, Sample{});
        else pass(uint32_t{}, Sample{});
        hipLaunchKernelGGL(k_one_root, dim3(1), dim3(kRootThreads), 0, st, parent, n, roots);
        if (dt == F32) pass(float{}, Rest{});
        else pass(uint32_t{}, Rest{});
    }
    hipLaunchKernelGGL(k_features_finish, dim3(1), dim3(kFinishThreads), 0, st, parent, n > 1 ? n : 0, 1, edges, x);
    return hipGetLastError();
}

}  // namespace apsp
