// Internal declarations shared by the HIP translation units of libapsp.
// Not installed; the public interface is include/apsp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_plan.h"

namespace apsp {

// I32P16: int32 data whose min-plus products run in capped 16-bit arithmetic
// (internal; the public dtype stays int32).
enum DType : int32_t { I32 = 0, F32 = 1, I32P16 = 2 };

constexpr uint32_t kInfI32 = 1u << 30;
// Cap of the capped 16-bit min-plus mode: stands for "no path below the cap"
// (two capped values plus the pattern offsets stay a finite binary16 pattern).
constexpr uint32_t kCap16 = 0x39ffu;

// One min-plus product C <- min(C, A (min,+) B) over a rectangular window.
// Optional exclusion bands remove a run of tile rows / tile columns from the
// launch (blocked FW excludes the pivot band from its panel and remainder
// updates).  With ksplit > 1 the reduction dimension is cut into chunks of
// kchunk elements and the partial minima are merged with atomic min.
struct GemmProblem {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t skip_m0, skip_mc;   // first excluded tile row, number excluded
    int32_t skip_n0, skip_nc;   // first excluded tile column, number excluded
    int32_t tiles_m, tiles_n;   // tiles launched (after exclusion)
    int32_t ksplit, kchunk;
    int32_t wg_begin;           // first workgroup of this problem in the launch
    int32_t pad_;
};

constexpr int kMaxGroup = 2;

// Up to kMaxGroup independent products in one launch.
struct GemmGroup {
    GemmProblem p[kMaxGroup];
    int32_t count;
    int32_t total_wgs;
};

enum Tile : int32_t { TILE_128 = 1, TILE_64 = 2 };

struct TileShape { int mt, nt, kt; };
TileShape tile_shape(int tile, DType dt = I32);

// Fills tiles/wg fields of every problem and the group total for `tile`.
// split_target: desired number of workgroups (0 disables split-K).
void finalize_group(GemmGroup& g, int tile, int split_target, DType dt = I32);

// skip: reduction slices whose staged A or B values are all INF are not folded.
hipError_t launch_minplus(DType dt, int tile, const GemmGroup& g, bool skip, hipStream_t s);

// Closure of an s x s diagonal block (s <= 128) held at D (leading dim ld).
// kind: 1 = Eq. 1 k-loop, 2 = squaring to a fixpoint.
hipError_t launch_closure(DType dt, int kind, void* D, int64_t ld, int32_t s, hipStream_t st);
// Blocked FW pivot step fused: X <- min(X, Cp (min,+) Rp) over bk steps, then
// X <- X* (k-loop closure), one workgroup; w <= 128, bk <= 128; int32 data
// for I32 and I32P16.
hipError_t launch_pivot_fused(DType dt, void* X, int64_t ld, const void* Cp, const void* Rp, int32_t w,
                              int32_t bk, hipStream_t st);

// Counts contract violations into *d_count (uint64, pre-zeroed by the kernel
// launcher on the same stream).
hipError_t launch_validate(DType dt, const void* D, int64_t n, int64_t ld,
                           unsigned long long* d_count, hipStream_t st);

// Counts entries of the n x n int32 matrix that are >= thr into *d_count
// (uint64, zeroed by the caller on the same stream).
hipError_t launch_count_ge(const uint32_t* D, int64_t n, int64_t ld, uint32_t thr,
                           unsigned long long* d_count, hipStream_t st);

// Fill kernel used instead of hipMemsetAsync for small device counters.
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st);

// Issue-rate calibration: a spin kernel running the fold of `dt` (I32P16 =
// the capped 16-bit fold) for `iters` iterations per lane on registers.
struct FoldSpin {
    int instr;   // fold instructions per iteration and lane
    int terms;   // min-plus terms per iteration and lane
};
FoldSpin fold_spin_shape(DType dt);
int fold_spin_threads();
hipError_t launch_fold_spin(DType dt, int grid, int iters, uint32_t seed, uint32_t* sink, hipStream_t st);

// One min-plus squaring pass D <- min(D, D (min,+) D) with change detection:
// *d_changed is set to 1 when any entry decreased.
hipError_t launch_square_pass(DType dt, int tile, void* D, int64_t n, int64_t ld,
                              uint32_t* d_changed, bool skip, hipStream_t st);

// Whole-graph squaring of an n x n int32 or fp32 matrix in one launch (n
// small enough that the passes are latency-bound); sync: the
// kSquareSyncWords words of tickets, pass counters and flags (zeroed here by
// a fill kernel); sync[49] receives an error bit if a wait overran and
// sync[50] the number of passes run.
constexpr int kSquareSyncWords = 64;
hipError_t launch_square_flow(DType dt, void* D, int n, int64_t ld, uint32_t* sync, int num_cus, hipStream_t st);

// Ragged batch: graph g is the n x n row-major matrix at data + offsets[g]
// (elements), n = sizes[g].  Workgroups take graphs in the order order[0..count).
struct BatchArgs {
    void* data;
    const int64_t* offsets;
    const int32_t* sizes;
    const int32_t* order;
    int32_t count;
    uint32_t* counter;   // ticket counter, zeroed by launch_batched
};

// Device record of the batch buffers read by the lock-step kernels.
struct BatchPtrs {
    void* data;
    const int64_t* offsets;
    const int32_t* sizes;
};
hipError_t launch_batch_ptrs(BatchPtrs* bp, void* data, const int64_t* offsets, const int32_t* sizes,
                             hipStream_t st);
// phase 0: pivot closures; 1: panel tiles; 3: remainder update of the next
// pivot tile (r+1, r+1) followed by its closure; 4: the other remainder
// tiles on 64 x 64 sub-tiles, sub-tile (si, sj) in bits 8 and 9 of the round
// (items: int4 {graph, round, a, b}).  Other phases: hipErrorInvalidValue.
hipError_t launch_batch_phase(DType dt, int phase, const BatchPtrs* bp, const int4* items, int count,
                              hipStream_t st);
int batched_round_width();

// Zeroes the per-XCD tickets and counters[0..ncounters), then launches
// nxcd * qlen_max workgroups; queue x holds tasks[qoff[x] .. qoff[x+1]);
// *err gets bit 0 if a wait overran.  global: the tasks of one queue run on
// every XCD (nxcd = 1 on a device with several), so each task releases its
// stores at agent scope before it signals.
hipError_t launch_batch_queue(DType dt, const BatchPtrs* bp, const BatchTask* tasks, const int32_t* qoff, int nxcd,
                              int qlen_max, uint32_t* tickets, int32_t* counters, int ncounters, uint32_t* err,
                              bool global, hipStream_t st);
// Finite off-diagonal entries of every graph of a batch, summed into *total
// (uint64, zeroed first).
hipError_t launch_batch_edges(DType dt, const void* data, const int64_t* offsets, const int32_t* sizes, int count,
                              unsigned long long* total, hipStream_t st);
// 32-bit words of ticket space for nxcd queues (one 256-byte slot each).
int batch_queue_ticket_words(int nxcd);
int batch_queue_resident_per_cu(DType dt);

// Enqueues the counter reset and the persistent batched kernel.
hipError_t launch_batched(DType dt, const BatchArgs& a, int grid, hipStream_t st);
int batched_resident_per_cu(DType dt);
const void* batched_kernel(DType dt);
int batched_max_n();        // lock-step and persistent schedules
constexpr int kQueueMaxN = 8192;   // queue schedule

// ---- last-hop predecessors (pred.hip)
// Sparse last-hop predecessors: column ranges of 1024, edges packed as
// v | (j - range start) << 16 | cost bits << 32, ordered by v within a range.
// launch_edge_count fills counts[r * n + v] (edges of row v in range r);
// launch_edge_scan turns them into offsets[r * n + v], range starts at
// offsets[cells + r] (cells = ranges * n) and the total at
// offsets[cells + ranges], and sets *use_sparse = (m <= edge_cap &&
// m <= dense_limit); launch_pred_sparse (skipped when !*use_sparse) writes
// the edges and then P.  n <= 65535.
int pred_sparse_ranges(int32_t n);
hipError_t launch_edge_count(DType dt, const void* W, int64_t ldw, int32_t n, int32_t* counts, hipStream_t st);
hipError_t launch_edge_scan(const int32_t* counts, int32_t n, int64_t* offsets, int64_t edge_cap,
                            int64_t dense_limit, uint32_t* use_sparse, hipStream_t st);
hipError_t launch_pred_sparse(DType dt, const void* D, int64_t ldd, const void* W, int64_t ldw, int32_t* P,
                              int64_t ldp, int32_t n, const int64_t* offsets, const int64_t* range_start,
                              uint64_t* edges, const uint32_t* use_sparse, hipStream_t st);
// Walks P back from dst[q] to src[q] for count queries (see apsp_path).
hipError_t launch_paths(const int32_t* P, int64_t ldp, int32_t n, int32_t count, const int32_t* src,
                        const int32_t* dst, int32_t* paths, int32_t max_len, int32_t* len, hipStream_t st);
// Dense argmin form; returns at once when skip_if_set is non-NULL and *skip_if_set != 0.
hipError_t launch_predecessors(DType dt, const void* D, int64_t ldd, const void* W, int64_t ldw, int32_t* P,
                               int64_t ldp, int32_t n, const uint32_t* skip_if_set, hipStream_t st);

// ---- planner features (features.hip)
// Edge count and weak connectivity of an n x n cost matrix: *edges (uint64)
// and *roots (uint32: the sampled pass's one-root flag) are zeroed first,
// parent (n int32) is a union-find forest in the workspace; x[0..3]
// receives the cost model's inputs (log2 n, log10 density, log2 batch = 0,
// connected).
hipError_t launch_graph_features(DType dt, const void* D, int32_t n, int64_t ld, int32_t* parent,
                                 unsigned long long* edges, uint32_t* roots, float* x, hipStream_t st);

// ---- cost-model MLP (mlp.hip)
constexpr int kMlpIn = 4;
constexpr int kMlpHidden = 64;
__host__ __device__ constexpr int mlp_param_count(int K)
{
    return kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden * K + K;
}
// floats of activation workspace for `rows` rows
__host__ __device__ constexpr int64_t mlp_workspace_floats(int rows, int K)
{
    return (int64_t)rows * (6 * kMlpHidden + K);
}
struct MlpNorm {
    float mu[kMlpIn];
    float sd[kMlpIn];
};
struct MlpAdam {
    float lr, beta1, beta2, eps;
    int32_t t0;   // Adam steps already taken (bias-correction offset)
};
hipError_t launch_mlp_forward(const float* P, const MlpNorm& nm, const float* X, int rows, int K, float* ws,
                              float* out, hipStream_t st);
hipError_t launch_mlp_train(float* P, float* M, float* V, const MlpNorm& nm, const float* X, const float* T,
                            const float* Msk, int rows, int K, int steps, const MlpAdam& opt, float* ws, float* G,
                            float* losses, hipStream_t st);
hipError_t launch_argmin_rows(const float* out, int rows, int K, int32_t* choice, hipStream_t st);

}  // namespace apsp
