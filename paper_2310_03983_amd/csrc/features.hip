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
// grandparent (again only by compare-and-swap).  A second pass counts the
// roots: the graph is weakly connected iff there is exactly one.
#include "internal.h"

#include <algorithm>

namespace apsp {

namespace {

constexpr int kThreads = 256;

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

__device__ __forceinline__ void unite(int32_t* parent, int32_t a, int32_t b)
{
    int32_t ra = find_root(parent, a), rb = find_root(parent, b);
    while (ra != rb) {
        if (ra > rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        // hook the larger root rb under ra, if rb is still a root
        const int32_t old = atomicCAS(parent + rb, rb, ra);
        if (old == rb) return;
        rb = find_root(parent, old);   // rb was hooked meanwhile: continue from its new root
        ra = find_root(parent, ra);
    }
}

template <class T>
__device__ __forceinline__ bool edge(T w);
template <>
__device__ __forceinline__ bool edge<uint32_t>(uint32_t w) { return w < kInfI32; }
template <>
__device__ __forceinline__ bool edge<float>(float w) { return w < __builtin_inff(); }

__global__ __launch_bounds__(kThreads) void k_parent_init(int32_t* parent, int32_t n)
{
    for (int32_t v = blockIdx.x * kThreads + threadIdx.x; v < n; v += gridDim.x * kThreads) parent[v] = v;
}

// Rows are taken by workgroups; the row's root is found once, and an edge
// whose other end already has that vertex as its parent is in the same tree
// (both ends hang below it) and skips the union.
template <class T>
__global__ __launch_bounds__(kThreads) void k_graph_edges(const T* __restrict__ D, int32_t n, int64_t ld,
                                                          int32_t* parent, unsigned long long* edges)
{
    uint32_t cnt = 0;
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const T* row = D + (int64_t)i * ld;
        const int32_t ri = find_root(parent, i);
        for (int32_t j = threadIdx.x; j < n; j += kThreads) {
            if (j == i || !edge<T>(row[j])) continue;
            ++cnt;
            if (load_parent(parent, j) == ri) continue;
            unite(parent, ri, j);
        }
    }
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

__global__ __launch_bounds__(kThreads) void k_count_roots(int32_t* parent, int32_t n, uint32_t* roots)
{
    uint32_t cnt = 0;
    for (int32_t v = blockIdx.x * kThreads + threadIdx.x; v < n; v += gridDim.x * kThreads)
        cnt += load_parent(parent, v) == v;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(roots, cnt);
}

// The cost model's inputs: log2 n, log10 density (clamped to 1e-9),
// log2 batch, weakly connected (1 / 0).
__global__ void k_features_final(int32_t n, int32_t batch, const unsigned long long* edges, const uint32_t* roots,
                                 float* x)
{
    if (threadIdx.x != 0) return;
    const double pairs = (double)n * (double)(n > 1 ? n - 1 : 1);
    const double dens = fmax((double)*edges / pairs, 1e-9);
    x[0] = (float)log2((double)(n > 1 ? n : 1));
    x[1] = (float)log10(dens);
    x[2] = (float)log2((double)(batch > 1 ? batch : 1));
    x[3] = (n <= 1 || *roots == 1u) ? 1.f : 0.f;   // one vertex (or none) is connected
}

}  // namespace

hipError_t launch_graph_features(DType dt, const void* D, int32_t n, int64_t ld, int32_t* parent,
                                 unsigned long long* edges, uint32_t* roots, float* x, hipStream_t st)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(edges), 0u, 2, st);
    if (e == hipSuccess) e = launch_fill_u32(roots, 0u, 1, st);
    if (e != hipSuccess) return e;
    if (n > 1) {
        const int gi = (int)std::min<int64_t>((n + kThreads - 1) / kThreads, 1024);
        const int gr = (int)std::min<int64_t>(n, 4096);
        hipLaunchKernelGGL(k_parent_init, dim3(gi), dim3(kThreads), 0, st, parent, n);
        if (dt == F32)
            hipLaunchKernelGGL(k_graph_edges<float>, dim3(gr), dim3(kThreads), 0, st, (const float*)D, n, ld, parent,
                               edges);
        else
            hipLaunchKernelGGL(k_graph_edges<uint32_t>, dim3(gr), dim3(kThreads), 0, st, (const uint32_t*)D, n, ld,
                               parent, edges);
        hipLaunchKernelGGL(k_count_roots, dim3(gi), dim3(kThreads), 0, st, parent, n, roots);
    }
    hipLaunchKernelGGL(k_features_final, dim3(1), dim3(64), 0, st, n, 1, edges, roots, x);
    return hipGetLastError();
}

}  // namespace apsp
