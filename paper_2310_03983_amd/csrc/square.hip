// Whole-graph min-plus squaring (Sec. 3.2) of a small graph in one launch.
// The passes D <- min(D, D (min,+) D) are cut into tasks, one output tile of
// one pass each (64 x 64, or 32 x 32 when the 64-tiles would leave most CUs
// idle; each task reads its row and column strips and folds the whole
// reduction, so one workgroup lowers and writes the tile and reports any
// decrease in the pass's "changed" word).  Workgroups take tickets in pass
// order from one counter and loop until the tickets run out.  A task of
// pass p waits until every task of pass p - 1 has signalled its pass
// counter: all of those hold smaller tickets, and a workgroup holding a
// ticket is running, so every wait ends whether or not the grid fits on the
// device at once (no cooperative launch, whose start costs more than a
// pass here).  When pass p - 1 changed nothing, D is closed: the task
// records the convergence and skips, and every later task skips without
// waiting.  At most ceil(log2(n - 1)) passes run, by which every shortest
// path (at most n - 1 edges) is covered.  The counters live in the context
// scratch and are zeroed by a fill kernel before the launch.
//
// Updates are in place: a pass may read entries that other tasks have
// already lowered.  Every stored value stays the length of a real walk and
// entries only decrease, so a pass ends at or below the out-of-place pass
// and the fixpoint is the same closure (int32 exact; fp32 within rounding).
//
// Coherence across XCDs: a task waits for its stores, then takes an
// agent-scope release (its tile becomes visible device-wide) before it
// increments its pass counter; a waiting task takes an agent-scope acquire
// after the counter is complete, before it reads.  Counters and flags are
// atomics at agent scope.
#include "device.h"
#include "internal.h"

#include <algorithm>

namespace apsp {

namespace {

constexpr int kSqThreads = 256;
constexpr uint32_t kSpinLimit = 1u << 22;

// Words of the synchronisation block (uint32 indices): the ticket counter,
// one done counter and one "changed" word per pass (at most 16 passes), the
// convergence word (~p once pass p is known to be a no-op, 0 before), the
// error word and the number of passes run.
constexpr int kSyncTicket = 0, kSyncDone = 16, kSyncChanged = 32, kSyncConv = 48, kSyncErr = 49, kSyncPasses = 50;
constexpr int kMaxPasses = 16;

__device__ __forceinline__ uint32_t rmw_read(uint32_t* p)
{
    return __hip_atomic_fetch_add(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class S, int TILE>
__global__ __launch_bounds__(kSqThreads) void k_square_flow(typename S::T* D, int64_t ld, int n, int tiles,
                                                            int max_passes, uint32_t* sync)
{
    using P = typename S::P;
    constexpr int TM = TILE / 16;   // 16 x 16 lanes, TM x TM entries each
    // reduction steps per staged slice: the small tiles' few slices are
    // latency-bound, so they take longer slices
    constexpr int kSqKT = TILE == 32 ? 64 : 32;
    __shared__ P As[2][kSqKT / S::KPACK][TILE + 2];
    __shared__ P Bs[2][kSqKT / S::KPACK][TILE + 2];
    __shared__ int s_ticket;
    __shared__ int s_run;
    const int tasks = tiles * tiles;
    const int total = tasks * max_passes;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (int)atomicAdd(sync + kSyncTicket, 1u);
        __syncthreads();
        const int tk = s_ticket;
        if (tk >= total) break;   // the same for every lane
        const int pass = tk / tasks, t = tk - pass * tasks;
        if (threadIdx.x == 0) {
            int run = 1;
            if (pass > 0) {
                uint32_t* done = sync + kSyncDone + pass - 1;
                uint32_t polls = 0;
                for (;;) {
                    const uint32_t conv = rmw_read(sync + kSyncConv);
                    if (conv != 0 && (int)~conv <= pass) {   // converged before this pass
                        run = 0;
                        break;
                    }
                    if (rmw_read(done) >= (uint32_t)tasks) break;
                    if (++polls > kSpinLimit) {   // cannot happen (see above); never hang
                        atomicOr(sync + kSyncErr, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (run) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    if (rmw_read(sync + kSyncChanged + pass - 1) == 0) {   // pass - 1 changed nothing
                        atomicMax(sync + kSyncConv, ~(uint32_t)pass);
                        run = 0;
                    }
                }
            }
            s_run = run;
        }
        __syncthreads();
        if (s_run) {
            const int tm = t / tiles, tn = t - tm * tiles;
            dev::mp_tile<S, TILE, TILE, kSqKT, TM, TM, true>(D, ld, D, ld, D, ld, n, n, tm * TILE, tn * TILE, 0, n,
                                                            false, sync + kSyncChanged + pass, As, Bs);
            __builtin_amdgcn_s_waitcnt(0);   // this lane's stores and flag update are done
            __syncthreads();
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(sync + kSyncDone + pass, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t == 0) atomicMax(sync + kSyncPasses, (uint32_t)(pass + 1));
            }
        }
        // a skipped task signals nothing: every later task skips too
        __syncthreads();   // s_ticket and the staging buffers are reused
    }
}

template <class S, int TILE>
hipError_t launch_flow(void* D, int n, int64_t ld, uint32_t* sync, int num_cus, hipStream_t st)
{
    int tiles = (n + TILE - 1) / TILE;
    static const int per_cu = [] {
        int b = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_square_flow<S, TILE>, kSqThreads, 0) == hipSuccess
                   ? b
                   : 0;
    }();
    const int grid = std::min(tiles * tiles, std::max(per_cu, 1) * num_cus);
    int max_passes = 0;
    while ((int64_t{1} << max_passes) < (int64_t)n - 1) ++max_passes;
    if (max_passes > kMaxPasses) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(sync, 0u, kSquareSyncWords, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_square_flow<S, TILE>), dim3(grid), dim3(kSqThreads), 0, st,
                       static_cast<typename S::T*>(D), ld, n, tiles, max_passes, sync);
    return hipGetLastError();
}

template <class S>
hipError_t launch_flow_sem(void* D, int n, int64_t ld, uint32_t* sync, int num_cus, hipStream_t st)
{
    const int t64 = (n + 63) / 64;
    if (t64 * t64 >= num_cus) return launch_flow<S, 64>(D, n, ld, sync, num_cus, st);
    return launch_flow<S, 32>(D, n, ld, sync, num_cus, st);
}

}  // namespace

hipError_t launch_square_flow(DType dt, void* D, int n, int64_t ld, uint32_t* sync, int num_cus, hipStream_t st)
{
    if (n <= 2) return hipSuccess;   // one edge is the shortest path between two vertices
    if (dt == F32) return launch_flow_sem<dev::SemF32>(D, n, ld, sync, num_cus, st);
    if (dt == I32) return launch_flow_sem<dev::SemI32>(D, n, ld, sync, num_cus, st);
    return hipErrorInvalidValue;
}

}  // namespace apsp
