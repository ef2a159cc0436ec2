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

template <class S>
__global__ void k_validate(const typename S::T* __restrict__ D, int64_t n, int64_t ld,
                           unsigned long long* __restrict__ count);

template <>
__global__ void k_validate<CI32>(const uint32_t* __restrict__ D, int64_t n, int64_t ld,
                                 unsigned long long* __restrict__ count)
{
    unsigned long long bad = 0;
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e - r * n;
        const uint32_t v = D[r * ld + c];   // negative int32 reads as > INF
        if (r == c ? v != 0u : v > kInfI32) ++bad;
    }
    if (bad) atomicAdd(count, bad);
}

template <>
__global__ void k_validate<CF32>(const float* __restrict__ D, int64_t n, int64_t ld,
                                 unsigned long long* __restrict__ count)
{
    unsigned long long bad = 0;
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e - r * n;
        const float v = D[r * ld + c];
        if (r == c ? !(v == 0.0f) : !(v >= 0.0f)) ++bad;   // NaN fails both tests
    }
    if (bad) atomicAdd(count, bad);
}

__global__ void k_count_ge(const uint32_t* __restrict__ D, int64_t n, int64_t ld, uint32_t thr,
                           unsigned long long* __restrict__ count)
{
    unsigned long long hits = 0;
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, c = e - r * n;
        if (D[r * ld + c] >= thr) ++hits;
    }
    if (hits) atomicAdd(count, hits);
}

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
    const int64_t total = n * n;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 2048);
    if (dt == I32)
        hipLaunchKernelGGL(k_validate<CI32>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const uint32_t*)D, n, ld, d_count);
    else
        hipLaunchKernelGGL(k_validate<CF32>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const float*)D, n, ld, d_count);
    return hipGetLastError();
}

hipError_t launch_count_ge(const uint32_t* D, int64_t n, int64_t ld, uint32_t thr,
                           unsigned long long* d_count, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t total = n * n;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(k_count_ge, dim3((unsigned)blocks), dim3(256), 0, st, D, n, ld, thr, d_count);
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
