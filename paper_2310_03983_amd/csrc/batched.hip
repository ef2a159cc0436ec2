// Many independent graphs of uneven sizes (a ragged batch) closed by blocked
// Floyd-Warshall (Sec. 2, Eq. 1) in one of three schedules:
//   the dependency-driven queue (k_bqueue, below): every pivot closure,
//     panel tile and remainder tile of every graph is a task of its own;
//   lock-step rounds (k_bclose, k_btile, k_bpivot, k_bsub): all graphs
//     advance one 128-wide round per group of launches;
//   one persistent kernel (k_batched, this first part).
//
// Persistent kernel: every workgroup repeatedly takes the next graph from a
// queue (one atomic ticket counter; the queue is ordered largest-first on the
// host, so the long graphs start first and the small ones fill the tail) and
// solves that graph on its own:
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

// ---------------------------------------------------------------------------
// Dependency-driven schedule: one launch runs every task of every graph --
// first pivot closures, panel tiles, remainder tiles, fused next pivots of
// its Floyd-Warshall rounds -- from ticket queues, one queue per XCD.  A
// workgroup reads which XCD it runs on, takes the next ticket of that XCD's
// queue, waits until the counters its task depends on reach their targets,
// runs the task and increments its own counter.  All tasks of a graph are
// in one queue, so a tile is written and read through one L2: a producer
// only waits for its stores to complete before it signals (no write-back of
// the L2), and a consumer invalidates its CU's L1 before it reads.  Each queue lists its tasks in a
// topological order (every task a task waits for has a smaller ticket in
// the same queue) and a workgroup that holds a ticket is running, so every
// queue drains.  Waits are bounded: past kSpinLimit polls the workgroup
// records the overrun in the error word and runs the task anyway, so every
// launch ends.  The grid holds qlen_max workgroups per XCD (workgroups are
// dispatched to the XCDs in turn); a workgroup whose queue is empty returns.
// Global mode (one queue, nxcd = 1, for batches of a few large graphs): any
// workgroup takes the next ticket, a graph's tasks run on every XCD, and a
// producer writes its stores back beyond its L2 (agent-scope release)
// before it signals.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 20;
constexpr int kTicketStride = 64;   // one 256-byte slot per XCD queue

// Polls with an atomic read-modify-write (adding 0), which is performed
// where the producers' increments are: in this XCD's L2.
__device__ __forceinline__ void wait_counter(int32_t* c, int32_t need, uint32_t* err)
{
    uint32_t polls = 0;
    while (__hip_atomic_fetch_add(c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++polls > kSpinLimit) {
            atomicOr(err, 1u);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// One workgroup per task: each workgroup takes a ticket when it starts.
template <class S>
__global__ __launch_bounds__(dev::kCloseWideThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_bqueue(const BatchPtrs* __restrict__ bp, const BatchTask* __restrict__ tasks, const int32_t* __restrict__ qoff,
              int nxcd, uint32_t* tickets, int32_t* counters, uint32_t* err, int global)
{
    using T = typename S::T;
    using P = typename S::P;
    constexpr int KT = 16;
    constexpr int kTileBytes = 2 * 2 * (KT / 2) * (kB + 2) * (int)sizeof(P);
    constexpr int kBytes = kTileBytes > dev::kCloseLdsWords * 4 ? kTileBytes : dev::kCloseLdsWords * 4;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    __shared__ int slot;
    auto As = reinterpret_cast<P (*)[KT / 2][kB + 2]>(smem);
    auto Bs = reinterpret_cast<P (*)[KT / 2][kB + 2]>(smem + kTileBytes / 2);
    const int tid = threadIdx.x;
    if (tid == 0) {
        // XCC_ID (bits 3:0 of hardware register 20): the XCD this workgroup runs on
        const int x = (int)((unsigned)__builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) % (unsigned)nxcd);
        const int q0 = qoff[x], len = qoff[x + 1] - q0;
        const int tk = len > 0 ? (int)atomicAdd(tickets + x * kTicketStride, 1u) : 0;
        slot = tk < len ? q0 + tk : -1;
    }
    __syncthreads();
    const int q = slot;
    if (q < 0) return;
    const BatchTask t = tasks[q];
    if (tid == 0) {
        if (t.wait0 >= 0) wait_counter(counters + t.wait0, t.need0, err);
        if (t.wait1 >= 0) wait_counter(counters + t.wait1, t.need1, err);
        // the inputs were written on this XCD and sit in its L2; an
        // agent-scope acquire drops the older copies this CU's L1 may hold
        // (an invalidation at workgroup scope would leave the L1 alone)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();   // every lane reads the task's inputs after the invalidation
    const int n = bp->sizes[t.graph];
    T* D = static_cast<T*>(bp->data) + bp->offsets[t.graph];
    const int64_t ld = n;
    const int W = t.width;              // the graph's round width: 64 or 128
    const int k0 = t.round * W, bk = min(W, n - k0);
    T* piv = D + (int64_t)k0 * ld + k0;
    // one product call site per width and one closure call site
    T* X = piv;   // block closed at the end (close and fused tasks)
    int w = bk;
    if (t.kind != kTaskClose) {
        const T* A;
        const T* B;
        T* C;
        int M, N;
        if (t.kind == kTaskRow) {            // R_KJ <- X* (min,+) R_KJ
            const int o0 = t.a * W;
            C = D + (int64_t)k0 * ld + o0;
            A = piv;
            B = C;
            M = bk;
            N = min(W, n - o0);
        } else if (t.kind == kTaskCol) {     // C_IK <- C_IK (min,+) X*
            const int o0 = t.a * W;
            C = D + (int64_t)o0 * ld + k0;
            A = C;
            B = piv;
            M = min(W, n - o0);
            N = bk;
        } else {                             // D_IJ <- min(D_IJ, C_IK (min,+) R_KJ); fused: (a, a)
            const int r0 = t.a * W, c0 = t.b * W;
            C = D + (int64_t)r0 * ld + c0;
            A = D + (int64_t)r0 * ld + k0;
            B = D + (int64_t)k0 * ld + c0;
            M = min(W, n - r0);
            N = min(W, n - c0);
            X = C;
            w = M;
        }
        if (t.sub >= 0) {
            // one 64 x 64 sub-tile (si, sj) of the tile: rows of C and A, columns of C and B
            const int si = (t.sub & 0xff) * 64, sj = (t.sub >> 8) * 64;
            C += (int64_t)si * ld + sj;
            A += (int64_t)si * ld;
            B += sj;
            M = min(64, M - si);
            N = min(64, N - sj);
        }
        if (W == kB && t.sub < 0)
            dev::mp_tile<S, kB, kB, KT, 8, 4, true>(A, ld, B, ld, C, ld, M, N, 0, 0, 0, bk, false, nullptr, As, Bs);
        else
            dev::mp_tile<S, 64, 64, 32, 4, 2, true>(A, ld, B, ld, C, ld, M, N, 0, 0, 0, bk, false, nullptr,
                                                   reinterpret_cast<P (*)[16][66]>(smem),
                                                   reinterpret_cast<P (*)[16][66]>(smem + 2 * 16 * 66 * sizeof(P)));
    }
    if (t.kind == kTaskClose || t.kind == kTaskFused) {
        // the fused task: round t.round's update of the next pivot block,
        // then the closure that starts round a
        __syncthreads();   // the block's stores are visible to the whole workgroup
        dev::close_block_wide<S>(X, ld, w, reinterpret_cast<T*>(smem));
    }
    __builtin_amdgcn_s_waitcnt(0);   // this lane's stores have reached the L2
    __syncthreads();                   // ... and every lane's
    if (tid == 0 && t.signal >= 0) {
        // one queue for the device: consumers may run on another XCD, so
        // the tile leaves this XCD's L2 before the counter moves
        if (global) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counters + t.signal, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// After the queue kernel: every queue must have handed out all its tickets.
// The grid holds qlen_max workgroups per XCD and workgroups are dispatched
// to the XCDs in turn, so each queue meets at least its length in
// workgroups; were a dispatch ever to leave one short, its last tasks would
// be skipped silently, so the shortfall is reported in bit 1 of *err.
__global__ void k_bqueue_claimed(const uint32_t* tickets, const int32_t* qoff, int nxcd, uint32_t* err)
{
    const int x = threadIdx.x;
    if (x < nxcd && tickets[x * kTicketStride] < (uint32_t)(qoff[x + 1] - qoff[x])) atomicOr(err, 2u);
}

// Edges of every graph of a batch (finite off-diagonal entries), summed into
// *total: one workgroup per graph (the batch planner's density input).
template <class T>
__device__ __forceinline__ bool finite_entry(T v);
template <>
__device__ __forceinline__ bool finite_entry<uint32_t>(uint32_t v) { return v < kInfI32; }
template <>
__device__ __forceinline__ bool finite_entry<float>(float v) { return v < __builtin_inff(); }

template <class T>
__global__ __launch_bounds__(256) void k_batch_edges(const T* __restrict__ data, const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ sizes,
                                                     unsigned long long* __restrict__ total)
{
    const int g = blockIdx.x;
    const int n = sizes[g];
    const T* D = data + offsets[g];
    const int nn = n * n;   // n <= 1024 in a batch
    uint32_t cnt = 0;
    for (int e = threadIdx.x; e < nn; e += 256) {
        const int r = e / n, c = e - r * n;
        cnt += (r != c) && finite_entry<T>(D[e]);
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(total, (unsigned long long)cnt);
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

hipError_t launch_batch_queue(DType dt, const BatchPtrs* bp, const BatchTask* tasks, const int32_t* qoff, int nxcd,
                              int qlen_max, uint32_t* tickets, int32_t* counters, int ncounters, uint32_t* err,
                              bool global, hipStream_t st)
{
    if (qlen_max <= 0) return hipSuccess;
    // tickets and counters start at zero on every launch (fill kernels, so
    // the sequence can be captured in a graph)
    hipError_t e = launch_fill_u32(tickets, 0u, (int64_t)nxcd * kTicketStride, st);
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(counters), 0u, ncounters, st);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)nxcd * (unsigned)qlen_max;
    if (dt == I32)
        hipLaunchKernelGGL(k_bqueue<dev::SemI32>, dim3(grid), dim3(dev::kCloseWideThreads), 0, st, bp, tasks, qoff,
                           nxcd, tickets, counters, err, global ? 1 : 0);
    else
        hipLaunchKernelGGL(k_bqueue<dev::SemF32>, dim3(grid), dim3(dev::kCloseWideThreads), 0, st, bp, tasks, qoff,
                           nxcd, tickets, counters, err, global ? 1 : 0);
    hipLaunchKernelGGL(k_bqueue_claimed, dim3(1), dim3(64), 0, st, tickets, qoff, nxcd, err);
    return hipGetLastError();
}

int batch_queue_ticket_words(int nxcd) { return nxcd * kTicketStride; }

int batch_queue_resident_per_cu(DType dt)
{
    int blocks = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, dt == I32 ? reinterpret_cast<const void*>(&k_bqueue<dev::SemI32>)
                           : reinterpret_cast<const void*>(&k_bqueue<dev::SemF32>),
        dev::kCloseWideThreads, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

hipError_t launch_batch_edges(DType dt, const void* data, const int64_t* offsets, const int32_t* sizes, int count,
                              unsigned long long* total, hipStream_t st)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(total), 0u, 2, st);
    if (e != hipSuccess || count <= 0) return e;
    if (dt == F32)
        hipLaunchKernelGGL(k_batch_edges<float>, dim3(count), dim3(256), 0, st, (const float*)data, offsets, sizes,
                           total);
    else
        hipLaunchKernelGGL(k_batch_edges<uint32_t>, dim3(count), dim3(256), 0, st, (const uint32_t*)data, offsets,
                           sizes, total);
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
