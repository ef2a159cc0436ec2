// Closure of one diagonal block (at most 128 x 128) inside a single
// workgroup: the base case of both blocked Floyd-Warshall (the pivot tile of
// every round) and R-Kleene (its leaves).
//
// k-loop (Sec. 2, Eq. 1): d[i][j] <- min(d[i][j], d[i][k] + d[k][j]) for
// k = 0..s-1, evaluated in the standard blocked order (pivot band, panels,
// remainder) so that most of the work uses the two-term packed fold; see
// k_closure_kloop below.
//
// Squaring (Sec. 3.2 applied to the block): X <- min(X, X (min,+) X) until no
// entry changes.  X lives in LDS; each pass computes the new 8 x 8 values in
// registers, then writes them back after a barrier.
#include "device.h"

#include <algorithm>

namespace apsp {

namespace {

using dev::kMaxS;
using CI32 = dev::SemI32;
using CF32 = dev::SemF32;

template <class S>
__global__ __launch_bounds__(dev::kCloseWideThreads) void k_closure_kloop(typename S::T* __restrict__ D, int64_t ld,
                                                                          int s)
{
    __shared__ __attribute__((aligned(16))) typename S::T lds[dev::kCloseLdsWords];
    dev::close_block_wide<S>(D, ld, s, lds);
}

template <class S>
__global__ __launch_bounds__(256) void k_closure_square(typename S::T* __restrict__ D, int64_t ld, int s)
{
    using T = typename S::T;
    __shared__ T X[kMaxS][kMaxS + 1];
    __shared__ int any_change;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;

    for (int e = tid; e < kMaxS * kMaxS; e += 256) {
        const int r = e / kMaxS, c = e % kMaxS;
        X[r][c] = (r < s && c < s) ? D[(int64_t)r * ld + c] : S::inf();
    }
    __syncthreads();

    // at most ceil(log2(s-1)) + 1 passes are needed; the bound only guards
    // against a non-monotone input (negative costs), which the contract excludes
    for (int pass = 0; pass < 2 * kMaxS; ++pass) {
        if (tid == 0) any_change = 0;
        T x[8][8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) x[i][j] = X[ty + 16 * i][tx + 16 * j];
        for (int k = 0; k < s; ++k) {
            T cv[8], rv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cv[i] = X[ty + 16 * i][k];
#pragma unroll
            for (int j = 0; j < 8; ++j) rv[j] = X[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) x[i][j] = S::relax(x[i][j], cv[i], rv[j]);
        }
        __syncthreads();
        bool changed = false;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                T& dst = X[ty + 16 * i][tx + 16 * j];
                if (x[i][j] < dst) {
                    changed = true;
                    dst = x[i][j];
                }
            }
        if (changed) any_change = 1;
        __syncthreads();
        if (!any_change) break;
        __syncthreads();
    }

    for (int e = tid; e < s * s; e += 256) {
        const int r = e / s, c = e % s;
        D[(int64_t)r * ld + c] = X[r][c];
    }
}

// Row-wise counting pass over an n x n matrix (HBM-bound): workgroups take
// whole rows, every lane reads 16-byte vectors (four elements; any 4-byte
// aligned row start works), four vectors in flight per lane, and the
// per-lane counts are summed across the wave and the workgroup before one
// 64-bit atomic per workgroup.  Test::bad(v, diagonal) decides an element.
struct ValidI32 {
    using T = uint32_t;
    // a negative int32 reads as > INF
    static __device__ __forceinline__ bool bad(uint32_t v, bool diag) { return diag ? v != 0u : v > kInfI32; }
};
struct ValidF32 {
    using T = float;
    // NaN fails both tests
    static __device__ __forceinline__ bool bad(float v, bool diag) { return diag ? !(v == 0.0f) : !(v >= 0.0f); }
};
struct AtLeast {
    using T = uint32_t;
    uint32_t thr;
    __device__ __forceinline__ bool bad(uint32_t v, bool) const { return v >= thr; }
};

constexpr int kCountThreads = 256;

template <class Test>
__global__ __launch_bounds__(kCountThreads) void k_count_rows(const typename Test::T* __restrict__ D, int64_t n,
                                                              int64_t ld, Test test,
                                                              unsigned long long* __restrict__ count)
{
    using T = typename Test::T;
    using V = dev::Pair2<dev::Pair2<T>>;   // four elements, one dwordx4 access
    constexpr int kStep = 4 * kCountThreads;          // elements per vector round
    uint32_t hits = 0;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const T* row = D + r * ld;
        int64_t c = (int64_t)threadIdx.x * 4;
        for (; c + 3 * kStep + 3 < n; c += 4 * kStep) {
            V v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = dev::ld_vec<V>(row + c + q * kStep);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t c0 = c + q * kStep;
                hits += test.bad(v[q].x.x, c0 == r) + test.bad(v[q].x.y, c0 + 1 == r) +
                        test.bad(v[q].y.x, c0 + 2 == r) + test.bad(v[q].y.y, c0 + 3 == r);
            }
        }
        for (; c + 3 < n; c += kStep) {
            const V v = dev::ld_vec<V>(row + c);
            hits += test.bad(v.x.x, c == r) + test.bad(v.x.y, c + 1 == r) + test.bad(v.y.x, c + 2 == r) +
                    test.bad(v.y.y, c + 3 == r);
        }
        for (; c < n; ++c) hits += test.bad(row[c], c == r);
    }
    // wave sum, then workgroup sum through LDS
    for (int off = 32; off > 0; off >>= 1) hits += __shfl_xor(hits, off);
    __shared__ uint32_t part[kCountThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = hits;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kCountThreads / 64; ++w) tot += part[w];
        if (tot) atomicAdd(count, tot);
    }
}

int count_grid(int64_t n) { return (int)std::min<int64_t>(n, 4096); }

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

// Next pivot of a blocked Floyd-Warshall round, fused in one 512-lane
// workgroup: the round's update of the pivot block from its two panel blocks,
// X <- min(X, Cp (min,+) Rp) over bk reduction steps (Sec. 2, Eq. 1 with k
// in the round's band), then the closure X <- X* (the next round's pivot
// step).  X, Cp and Rp are disjoint blocks of one matrix with stride ld.
template <class S>
__global__ __launch_bounds__(dev::kCloseWideThreads) void k_pivot_fused(typename S::T* X, int64_t ld,
                                                                        const typename S::T* __restrict__ Cp,
                                                                        const typename S::T* __restrict__ Rp, int w,
                                                                        int bk)
{
    using T = typename S::T;
    using P = typename S::P;
    constexpr int KT = 16;
    constexpr int kTileBytes = 2 * 2 * (KT / 2) * (kMaxS + 2) * (int)sizeof(P);
    constexpr int kBytes = kTileBytes > dev::kCloseLdsWords * 4 ? kTileBytes : dev::kCloseLdsWords * 4;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    auto As = reinterpret_cast<P (*)[KT / 2][kMaxS + 2]>(smem);
    auto Bs = reinterpret_cast<P (*)[KT / 2][kMaxS + 2]>(smem + kTileBytes / 2);
    dev::mp_tile<S, kMaxS, kMaxS, KT, 8, 4, true>(Cp, ld, Rp, ld, X, ld, w, w, 0, 0, 0, bk, false, nullptr, As, Bs);
    __syncthreads();   // the block's stores are visible to the whole workgroup
    dev::close_block_wide<S>(X, ld, w, reinterpret_cast<T*>(smem));
}

}  // namespace

hipError_t launch_closure(DType dt, int kind, void* D, int64_t ld, int32_t s, hipStream_t st)
{
    if (s <= 0) return hipSuccess;
    if (kind == 2) {
        if (dt == I32)
            hipLaunchKernelGGL(k_closure_square<CI32>, dim3(1), dim3(256), 0, st, (uint32_t*)D, ld, s);
        else
            hipLaunchKernelGGL(k_closure_square<CF32>, dim3(1), dim3(256), 0, st, (float*)D, ld, s);
    } else {
        if (dt == I32)
            hipLaunchKernelGGL(k_closure_kloop<CI32>, dim3(1), dim3(dev::kCloseWideThreads), 0, st, (uint32_t*)D, ld, s);
        else
            hipLaunchKernelGGL(k_closure_kloop<CF32>, dim3(1), dim3(dev::kCloseWideThreads), 0, st, (float*)D, ld, s);
    }
    return hipGetLastError();
}

hipError_t launch_pivot_fused(DType dt, void* X, int64_t ld, const void* Cp, const void* Rp, int32_t w,
                              int32_t bk, hipStream_t st)
{
    if (w <= 0) return hipSuccess;
    if (dt == F32)
        hipLaunchKernelGGL(k_pivot_fused<CF32>, dim3(1), dim3(dev::kCloseWideThreads), 0, st, (float*)X, ld,
                           (const float*)Cp, (const float*)Rp, w, bk);
    else
        hipLaunchKernelGGL(k_pivot_fused<CI32>, dim3(1), dim3(dev::kCloseWideThreads), 0, st, (uint32_t*)X, ld,
                           (const uint32_t*)Cp, (const uint32_t*)Rp, w, bk);
    return hipGetLastError();
}

hipError_t launch_validate(DType dt, const void* D, int64_t n, int64_t ld,
                           unsigned long long* d_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)d_count, 0u, (int64_t)2);
    if (n <= 0) return hipGetLastError();
    if (dt == I32)
        hipLaunchKernelGGL(k_count_rows<ValidI32>, dim3(count_grid(n)), dim3(kCountThreads), 0, st,
                           (const uint32_t*)D, n, ld, ValidI32{}, d_count);
    else
        hipLaunchKernelGGL(k_count_rows<ValidF32>, dim3(count_grid(n)), dim3(kCountThreads), 0, st,
                           (const float*)D, n, ld, ValidF32{}, d_count);
    return hipGetLastError();
}

hipError_t launch_count_ge(const uint32_t* D, int64_t n, int64_t ld, uint32_t thr,
                           unsigned long long* d_count, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_rows<AtLeast>, dim3(count_grid(n)), dim3(kCountThreads), 0, st, D, n, ld,
                       AtLeast{thr}, d_count);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
    return hipGetLastError();
}

}  // namespace apsp
