// Many independent graphs of uneven sizes closed in one persistent launch.
//
// Every workgroup repeatedly takes the next graph from a queue (one atomic
// ticket counter; the queue is ordered largest-first on the host, so the long
// graphs start first and the small ones fill the tail) and solves that graph
// on its own:
//   n <= 128: the whole matrix is closed in LDS by the block closure;
//   n  > 128: blocked Floyd-Warshall (Sec. 2, Eq. 1) with 128-wide rounds --
//            pivot closure, row/column panel tiles, remainder tiles -- all by
//            the same workgroup, operands streaming through L2.
// Workgroups never wait on each other, so the kernel cannot deadlock however
// many of them are resident; the grid is sized to the resident capacity.
#include "device.h"

#include <algorithm>

namespace apsp {

namespace {

using dev::kMaxS;

constexpr int kB = 128;                                  // round width
constexpr int kLdsClose = dev::kCloseLdsWords * 4;       // closure band buffers
constexpr int kLdsTile = 2 * 2 * (16 / 2) * (kB + 2) * 8; // A and B staging (pairs)
constexpr int kLds = kLdsClose > kLdsTile ? kLdsClose : kLdsTile;

// One graph, one workgroup.  Written with a single call site for the block
// closure and a single call site for the tile product (each inlined once):
// the work of a round is a list -- panel tiles first, then, after a barrier,
// remainder tiles -- walked by one loop.
template <class S, bool VEC>
__device__ __forceinline__ void solve_graph(typename S::T* D, int n, char* smem)
{
    using T = typename S::T;
    using P = typename S::P;
    T* X = reinterpret_cast<T*>(smem);
    auto As = reinterpret_cast<P (*)[8][kB + 2]>(smem);
    auto Bs = reinterpret_cast<P (*)[8][kB + 2]>(smem + 2 * 8 * (kB + 2) * sizeof(P));
    const int64_t ld = n;
    const int nt = (n + kB - 1) / kB;     // n <= 128 is a single round with no tiles
    for (int kt = 0; kt < nt; ++kt) {
        const int k0 = kt * kB;
        const int bk = min(kB, n - k0);
        T* piv = D + (int64_t)k0 * ld + k0;
        dev::close_block<S>(piv, ld, bk, X);
        __syncthreads();
        const int others = nt - 1;
        const int npanel = 2 * others;
        const int nitems = npanel + others * others;
        for (int it = 0; it < nitems; ++it) {
            if (it == npanel) __syncthreads();   // remainder reads the updated panels
            const T* A;
            const T* B;
            T* C;
            int M, N;
            if (it < npanel) {
                int t = it >> 1;
                t += (t >= kt);
                const int o0 = t * kB, w = min(kB, n - o0);
                if ((it & 1) == 0) {
                    // row panel R_KJ <- X* (min,+) R_KJ
                    A = piv;
                    B = D + (int64_t)k0 * ld + o0;
                    C = D + (int64_t)k0 * ld + o0;
                    M = bk;
                    N = w;
                } else {
                    // column panel C_IK <- C_IK (min,+) X*
                    A = D + (int64_t)o0 * ld + k0;
                    B = piv;
                    C = D + (int64_t)o0 * ld + k0;
                    M = w;
                    N = bk;
                }
            } else {
                // remainder D_IJ <- min(D_IJ, C_IK (min,+) R_KJ)
                const int r = it - npanel;
                int ti = r / others, tj = r - ti * others;
                ti += (ti >= kt);
                tj += (tj >= kt);
                const int r0 = ti * kB, c0 = tj * kB;
                A = D + (int64_t)r0 * ld + k0;
                B = D + (int64_t)k0 * ld + c0;
                C = D + (int64_t)r0 * ld + c0;
                M = min(kB, n - r0);
                N = min(kB, n - c0);
            }
            dev::mp_tile<S, kB, kB, 16, 8, 8, VEC>(A, ld, B, ld, C, ld, M, N, 0, 0, 0, bk, false, nullptr, As, Bs);
        }
        __syncthreads();
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_batched(BatchArgs a)
{
    using T = typename S::T;
    __shared__ __attribute__((aligned(16))) char smem[kLds];
    __shared__ int ticket;
    for (;;) {
        if (threadIdx.x == 0) ticket = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int q = ticket;
        __syncthreads();
        if (q >= a.count) break;
        const int g = a.order[q];
        const int n = a.sizes[g];
        T* D = static_cast<T*>(a.data) + a.offsets[g];
        const bool vec = (reinterpret_cast<uintptr_t>(D) & 3) == 0;
        if (vec)
            solve_graph<S, true>(D, n, smem);
        else
            solve_graph<S, false>(D, n, smem);
    }
}

// ---------------------------------------------------------------------------
// Lock-step schedule: every graph advances one 128-wide Floyd-Warshall round
// per wide launch group -- the pivot closures of all graphs, all their panel
// tiles, all their remainder tiles -- so a graph's tiles are spread over the
// whole device instead of one workgroup.  Work items are (graph, round, a,
// b): closure (a = b = 0); panel tile a of the row (b = 0) or column (b = 1)
// panel; remainder tile (a, b).  Graphs with n <= 128 are finished by their
// round-0 closure.  Data pointers are read from a small device record so
// that a captured launch sequence serves any buffers.  (The host orders the
// launches so that round r+1's pivot tiles and closures run on a second
// stream beside the rest of round r's remainder.)
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(dev::kCloseWideThreads) void k_bclose(const BatchPtrs* __restrict__ bp,
                                                                   const int4* __restrict__ items)
{
    using T = typename S::T;
    __shared__ __attribute__((aligned(16))) T lds[dev::kCloseLdsWords];
    const int4 it = items[blockIdx.x];
    const int n = bp->sizes[it.x];
    T* D = static_cast<T*>(bp->data) + bp->offsets[it.x];
    const int k0 = it.y * kB;
    dev::close_block_wide<S>(D + (int64_t)k0 * n + k0, n, min(kB, n - k0), lds);
}

// Panel tile update of round r (item (graph, r, t, b)): b = 0 the row panel
// R_KJ <- X* (min,+) R_KJ, b = 1 the column panel C_IK <- C_IK (min,+) X*,
// one 128 x 128 tile per workgroup.  The tile is read and written by the
// same workgroup (its reads finish before its epilogue stores), so the
// in-place update takes only the pre-update panel.
template <class S>
__global__ __launch_bounds__(256) void k_btile(const BatchPtrs* __restrict__ bp, const int4* __restrict__ items)
{
    using T = typename S::T;
    using P = typename S::P;
    __shared__ P As[2][8][kB + 2];
    __shared__ P Bs[2][8][kB + 2];
    const int4 it = items[blockIdx.x];
    const int n = bp->sizes[it.x];
    T* D = static_cast<T*>(bp->data) + bp->offsets[it.x];
    const int64_t ld = n;
    const int k0 = it.y * kB, bk = min(kB, n - k0);
    T* piv = D + (int64_t)k0 * ld + k0;
    const int o0 = it.z * kB, w = min(kB, n - o0);
    const T* A;
    const T* B;
    T* C;
    int M, N;
    if (it.w == 0) {            // row panel
        A = piv;
        C = D + (int64_t)k0 * ld + o0;
        B = C;
        M = bk;
        N = w;
    } else {                    // column panel
        C = D + (int64_t)o0 * ld + k0;
        A = C;
        B = piv;
        M = w;
        N = bk;
    }
    dev::mp_tile<S, kB, kB, 16, 8, 8, true>(A, ld, B, ld, C, ld, M, N, 0, 0, 0, bk, false, nullptr, As, Bs);
}

// Remainder update on 64 x 64 sub-tiles: item (graph, round | si << 8 |
// sj << 9, a, b) updates rows si*64.. and columns sj*64.. of tile (a, b).
// Four workgroups per 128-tile fill the device better than one at K = 128;
// the remainder reads only the pivot's row and column panels, which no
// remainder item writes, so the split changes no value.
template <class S>
__global__ __launch_bounds__(256) void k_bsub(const BatchPtrs* __restrict__ bp, const int4* __restrict__ items)
{
    using T = typename S::T;
    using P = typename S::P;
    constexpr int MT = 64, KT = 32;
    __shared__ P As[2][KT / 2][MT + 2];
    __shared__ P Bs[2][KT / 2][MT + 2];
    const int4 it = items[blockIdx.x];
    const int n = bp->sizes[it.x];
    T* D = static_cast<T*>(bp->data) + bp->offsets[it.x];
    const int64_t ld = n;
    const int r = it.y & 0xff;
    const int k0 = r * kB, bk = min(kB, n - k0);
    const int r0 = it.z * kB + ((it.y >> 8) & 1) * MT;
    const int c0 = it.w * kB + ((it.y >> 9) & 1) * MT;
    dev::mp_tile<S, MT, MT, KT, 4, 4, true>(D + (int64_t)r0 * ld + k0, ld, D + (int64_t)k0 * ld + c0, ld,
                                           D + (int64_t)r0 * ld + c0, ld, min(MT, n - r0), min(MT, n - c0), 0, 0,
                                           0, bk, false, nullptr, As, Bs);
}

// Next pivot of a graph: round r's remainder update of tile (r+1, r+1), then
// its closure, by one 512-lane workgroup (item (graph, r, r+1, r+1)).  No
// other remainder tile of round r reads or writes that block, so this runs
// beside them.
template <class S>
__global__ __launch_bounds__(dev::kCloseWideThreads) void k_bpivot(const BatchPtrs* __restrict__ bp,
                                                                   const int4* __restrict__ items)
{
    using T = typename S::T;
    using P = typename S::P;
    constexpr int KT = 16;
    constexpr int kTileBytes = 2 * 2 * (KT / 2) * (kB + 2) * (int)sizeof(P);
    constexpr int kBytes = kTileBytes > dev::kCloseLdsWords * 4 ? kTileBytes : dev::kCloseLdsWords * 4;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    auto As = reinterpret_cast<P (*)[KT / 2][kB + 2]>(smem);
    auto Bs = reinterpret_cast<P (*)[KT / 2][kB + 2]>(smem + kTileBytes / 2);
    const int4 it = items[blockIdx.x];
    const int n = bp->sizes[it.x];
    T* D = static_cast<T*>(bp->data) + bp->offsets[it.x];
    const int64_t ld = n;
    const int k0 = it.y * kB, bk = min(kB, n - k0);
    const int p0 = it.z * kB, w = min(kB, n - p0);
    T* X = D + (int64_t)p0 * ld + p0;
    dev::mp_tile<S, kB, kB, KT, 8, 4, true>(D + (int64_t)p0 * ld + k0, ld, D + (int64_t)k0 * ld + p0, ld, X, ld, w,
                                           w, 0, 0, 0, bk, false, nullptr, As, Bs);
    __syncthreads();   // the tile's stores are visible to the whole workgroup
    dev::close_block_wide<S>(X, ld, w, reinterpret_cast<T*>(smem));
}

__global__ void k_set_ptrs(BatchPtrs* bp, void* data, const int64_t* offsets, const int32_t* sizes)
{
    if (threadIdx.x == 0) {
        bp->data = data;
        bp->offsets = offsets;
        bp->sizes = sizes;
    }
}

}  // namespace

const void* batched_kernel(DType dt)
{
    return dt == I32 ? reinterpret_cast<const void*>(&k_batched<dev::SemI32>)
                     : reinterpret_cast<const void*>(&k_batched<dev::SemF32>);
}

int batched_max_n() { return 8 * kB; }

hipError_t launch_batched(DType dt, const BatchArgs& a, int grid, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    hipError_t e = launch_fill_u32(a.counter, 0u, 1, st);
    if (e != hipSuccess) return e;
    if (dt == I32)
        hipLaunchKernelGGL(k_batched<dev::SemI32>, dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_batched<dev::SemF32>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_ptrs(BatchPtrs* bp, void* data, const int64_t* offsets, const int32_t* sizes,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(64), 0, st, bp, data, offsets, sizes);
    return hipGetLastError();
}

hipError_t launch_batch_phase(DType dt, int phase, const BatchPtrs* bp, const int4* items, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (phase == 3) {
        if (dt == I32)
            hipLaunchKernelGGL(k_bpivot<dev::SemI32>, dim3(count), dim3(dev::kCloseWideThreads), 0, st, bp, items);
        else
            hipLaunchKernelGGL(k_bpivot<dev::SemF32>, dim3(count), dim3(dev::kCloseWideThreads), 0, st, bp, items);
        return hipGetLastError();
    }
    if (phase == 4) {
        if (dt == I32)
            hipLaunchKernelGGL(k_bsub<dev::SemI32>, dim3(count), dim3(256), 0, st, bp, items);
        else
            hipLaunchKernelGGL(k_bsub<dev::SemF32>, dim3(count), dim3(256), 0, st, bp, items);
        return hipGetLastError();
    }
    if (phase == 0) {
        if (dt == I32)
            hipLaunchKernelGGL(k_bclose<dev::SemI32>, dim3(count), dim3(dev::kCloseWideThreads), 0, st, bp, items);
        else
            hipLaunchKernelGGL(k_bclose<dev::SemF32>, dim3(count), dim3(dev::kCloseWideThreads), 0, st, bp, items);
    } else if (phase == 1) {
        if (dt == I32)
            hipLaunchKernelGGL(k_btile<dev::SemI32>, dim3(count), dim3(256), 0, st, bp, items);
        else
            hipLaunchKernelGGL(k_btile<dev::SemF32>, dim3(count), dim3(256), 0, st, bp, items);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int batched_round_width() { return kB; }

int batched_resident_per_cu(DType dt)
{
    int blocks = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, dt == I32 ? reinterpret_cast<const void*>(&k_batched<dev::SemI32>)
                           : reinterpret_cast<const void*>(&k_batched<dev::SemF32>),
        256, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

}  // namespace apsp
