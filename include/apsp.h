/*
 * apsp.h -- C ABI of the MI355X min-plus all-pairs-shortest-paths library.
 *
 * Method: T. Anjary, "The Floyd-Warshall Algorithm Re-implemented Using
 * 3D-Tensors and Hardware Acceleration", arXiv 2310.03983.
 *
 * Problem statement (Sec. 2 and Sec. 3.1):
 *   A graph on n vertices is given as a dense n x n cost matrix D, row-major
 *   with leading dimension ldd >= n elements; D[i*ldd + j] is the cost of the
 *   edge i -> j (row = "from" vertex, column = "to" vertex).  D[i][i] = 0
 *   (Sec. 3.4) and a missing edge holds INF.  Costs are non-negative.
 *   The solvers overwrite D in place with shortest-path distances.
 *
 * Element types (apsp_dtype_t):
 *   APSP_I32  int32 costs in [0, APSP_INF_I32]; APSP_INF_I32 = 2^30 means
 *             "no path".  Addition saturates: a (+) b = min(a + b, INF), so
 *             every result is exactly min(true distance, INF).
 *   APSP_F32  IEEE binary32 costs >= 0, +inf means "no path".  Each min-plus
 *             term is one round-to-nearest-even addition.
 *
 * Memory and streams: every matrix, offset and size array passed to a compute
 * call is device memory owned by the caller; the library keeps no pointer
 * past the call, except the workspace the caller registers with
 * apsp_set_workspace (kept until replaced or the context is destroyed).  No
 * compute call allocates or frees device memory: the only device memory a
 * call uses beyond its arguments is that workspace and the context's 4 KB
 * scratch (allocated by apsp_create).  `stream` is a hipStream_t (NULL = the
 * legacy default stream).  Compute calls only enqueue work and return unless
 * their comment says they synchronise; a device fault is reported by the
 * caller's next synchronisation.  Value preconditions (diagonal 0, range)
 * are not checked by compute calls; apsp_validate checks them.
 *
 * Errors: every call returns an apsp_status_t.  Argument errors are detected
 * before anything is enqueued.  apsp_last_error() returns a thread-local
 * message describing the last failure on the calling thread.
 *
 * Contexts: a context owns a second stream and three events (blocked FW's
 * look-ahead and the batched schedule fork work onto it and join back onto
 * the caller's stream before returning), a 4 KB device scratch, the cost
 * model's parameters and cached batched plans.  It is not thread-safe: use
 * it from one host thread at a time, and do not let calls through one
 * context run concurrently on different streams (create one context per
 * concurrent user).
 */
#ifndef APSP_H
#define APSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apsp_status_t;
#define APSP_OK             0
#define APSP_E_ARG         -1   /* null pointer, negative size, ld too small, bad dtype/option */
#define APSP_E_INPUT       -2   /* apsp_validate found a precondition violation */
#define APSP_E_NOMEM       -3   /* workspace missing or too small (apsp_workspace_size), or
                                   apsp_create could not allocate its scratch */
#define APSP_E_HIP         -4   /* a HIP runtime call or kernel launch failed */
#define APSP_E_UNSUPPORTED -5   /* option not available for this dtype/size */
#define APSP_E_STATE       -6   /* context not usable (wrong device, destroyed) */

typedef int32_t apsp_dtype_t;
#define APSP_I32 0
#define APSP_F32 1

#define APSP_INF_I32 1073741824  /* 2^30 */

/* Algorithm choice (apsp_opts_t.algo). */
#define APSP_ALGO_AUTO     0   /* planner decides */
#define APSP_ALGO_FW       1   /* three-phase blocked Floyd-Warshall (Sec. 2, Eq. 1) */
#define APSP_ALGO_RKLEENE  2   /* R-Kleene quadrant recursion (Sec. 3.3, Eq. 4) */
#define APSP_ALGO_SQUARE   3   /* min-plus squaring to a fixpoint (Sec. 3.2) */

/* Closure of a diagonal tile (apsp_opts_t.closure). */
#define APSP_CLOSURE_AUTO   0
#define APSP_CLOSURE_KLOOP  1  /* Eq. 1 k-loop held in LDS */
#define APSP_CLOSURE_SQUARE 2  /* X <- min(X, X (min,+) X) until unchanged (Sec. 3.2) */

/* GEMM macro-tile (apsp_opts_t.tile). */
#define APSP_TILE_AUTO    0
#define APSP_TILE_128     1   /* 128 x 128 output tile per workgroup */
#define APSP_TILE_64      2   /* 64 x 64 output tile per workgroup */

/* Flags (apsp_opts_t.flags). */
#define APSP_FLAG_NO_SPLITK        1  /* never split the reduction dimension */
#define APSP_FLAG_BATCH_NO_GRAPH   2  /* apsp_batched: launch directly, no HIP graph */
#define APSP_FLAG_BATCH_PER_GRAPH  4  /* apsp_batched: one launch per graph */
#define APSP_FLAG_NO_LOOKAHEAD     8  /* blocked FW: strictly sequential rounds on the caller's stream */
#define APSP_FLAG_BATCH_PERSISTENT 16 /* apsp_batched: one persistent kernel, one workgroup per graph */
#define APSP_FLAG_PACKED16         32 /* int32 apsp_fw / apsp_rkleene / apsp_square / apsp_solve:
                                         min-plus products in capped 16-bit arithmetic (see below) */
#define APSP_FLAG_BATCH_QUEUE      128 /* apsp_batched: dependency-driven schedule, one workgroup per task
                                          (see apsp_batched) */
#define APSP_FLAG_BATCH_LOCKSTEP   256 /* apsp_batched: the lock-step schedule (see apsp_batched) */
#define APSP_FLAG_BATCH_GLOBAL     512 /* apsp_batched with APSP_FLAG_BATCH_QUEUE: one ticket queue for the
                                          whole device instead of one per XCD (see apsp_batched) */
#define APSP_FLAG_DETERMINISTIC    1024 /* apsp_fw / apsp_rkleene / apsp_solve: results identical bit for bit
                                          from run to run (fp32; int32 results are unique anyway).  Every
                                          product whose output block is also one of its operands (R-Kleene's
                                          B <- A*B, C <- CA*, B <- BD*, C <- D*C; blocked FW's panels) reads
                                          a copy of that operand taken first, so no tile reads entries that
                                          other workgroups are lowering.  Needs a workspace of
                                          apsp_workspace_size(APSP_OP_DETERMINISTIC, n) (APSP_E_NOMEM
                                          otherwise); apsp_square rejects it (APSP_E_UNSUPPORTED). */
#define APSP_FLAG_SKIP_INF         64 /* minplus_gemm / apsp_fw / apsp_rkleene / apsp_square / apsp_solve:
                                         a product skips every reduction slice (16 or 32 steps of one
                                         tile) whose A block or B block is all INF -- exact, since
                                         C <= INF; pays off on very sparse graphs, costs a few
                                         instructions per slice otherwise.  apsp_closure and
                                         apsp_batched ignore it. */

typedef struct apsp_opts {
    int32_t algo;      /* APSP_ALGO_*; only apsp_solve and apsp_batched read it */
    int32_t block;     /* FW round width / R-Kleene leaf size: 0 (auto), 64 or 128; apsp_batched with
                          APSP_FLAG_BATCH_QUEUE: the round width of graphs with n > reserved[0] (others 128) */
    int32_t tile;      /* APSP_TILE_* for the min-plus products */
    int32_t closure;   /* APSP_CLOSURE_* for diagonal tiles */
    int32_t cutover;   /* R-Kleene: sub-problems <= cutover use blocked FW (0 = never) */
    int32_t flags;     /* APSP_FLAG_* bits */
    int32_t reserved[6];
} apsp_opts_t;

typedef struct apsp_ctx apsp_ctx_t;

/* Creates a context bound to HIP device `device` and allocates its 4 KB
 * device scratch (counters and flags).  *ctx receives the handle. */
apsp_status_t apsp_create(apsp_ctx_t **ctx, int32_t device);

/* Synchronises the device, frees the scratch and the handle.  NULL is a no-op. */
apsp_status_t apsp_destroy(apsp_ctx_t *ctx);

/* Thread-local text of the last error on this thread ("" if none). */
const char *apsp_last_error(void);

/* Library version string. */
const char *apsp_version(void);

/*
 * Workspace.  apsp_batched (its plan: queue order, work items, a pointer
 * record) and the sparse form of apsp_predecessors_ex (edge counts, offsets,
 * edge list) need device memory beyond their arguments; the caller provides
 * it once with apsp_set_workspace and the library never allocates it.
 * apsp_workspace_size returns the bytes an operation needs:
 *   APSP_OP_SOLVE         n_or_total = n: the feature pass of apsp_features
 *                         and of apsp_solve's cost-model plan (one int32 per
 *                         vertex; without it apsp_solve keeps the size
 *                         rule); apsp_fw / apsp_rkleene / apsp_square /
 *                         minplus_gemm / apsp_closure / apsp_validate need
 *                         no workspace;
 *   APSP_OP_BATCHED       n_or_total = the largest n of the batch, count = the
 *                         number of graphs: an upper bound for any batch of
 *                         that shape;
 *   APSP_OP_PREDECESSORS  n_or_total = n: the sparse form for every graph the
 *                         automatic choice takes sparse (up to n^2/4 edges);
 *                         0 for n > 65535 (dense only);
 *   APSP_OP_DETERMINISTIC n_or_total = n: the copies APSP_FLAG_DETERMINISTIC
 *                         takes for apsp_fw / apsp_rkleene / apsp_solve
 *                         (about n^2 / 2 elements for R-Kleene).
 * Returns 0 (and sets the last error) for an invalid context, dtype, op or
 * negative size.
 */
#define APSP_OP_SOLVE        0
#define APSP_OP_BATCHED      1
#define APSP_OP_PREDECESSORS 2
#define APSP_OP_DETERMINISTIC 3
size_t apsp_workspace_size(apsp_ctx_t *ctx, int32_t op, apsp_dtype_t dtype, int64_t n_or_total, int32_t count);

/*
 * Registers `bytes` of caller-owned device memory at d_ptr (256-byte
 * aligned; NULL with 0 clears it) as the context's workspace.  The library
 * keeps the pointer until it is replaced or the context is destroyed; the
 * caller keeps the memory alive that long and does not use it meanwhile.
 * Replacing a workspace drops the cached batched plans (they point into it)
 * after waiting for the device.  Every compute call that uses the workspace
 * overwrites it, so calls through one context that use it must not overlap.
 * Errors: APSP_E_ARG for a NULL pointer with bytes > 0 or a misaligned one.
 */
apsp_status_t apsp_set_workspace(apsp_ctx_t *ctx, void *d_ptr, size_t bytes);

/*
 * Min-plus product, accumulating form (Sec. 3, Eq. 2):
 *     C[i][j] <- min(C[i][j], min_{0<=t<k} A[i][t] (+) B[t][j])
 * A is m x k (lda >= k), B is k x n (ldb >= n), C is m x n (ldc >= n), all
 * row-major device arrays of `dtype`.  Filling C with INF first gives Eq. 2
 * exactly.  k = 0, m = 0 or n = 0 leaves C unchanged.  The result is exact
 * and unique in both dtypes (min is exact and each term is rounded once).
 * C must not overlap A or B (APSP_E_ARG).  Preconditions: A, B, C in
 * [0, INF] (int32) / >= 0 (fp32).
 */
apsp_status_t minplus_gemm(apsp_ctx_t *ctx, apsp_dtype_t dtype,
                           int64_t m, int64_t n, int64_t k,
                           const void *A, int64_t lda,
                           const void *B, int64_t ldb,
                           void *C, int64_t ldc,
                           const apsp_opts_t *opts, void *stream);

/*
 * Closure of one square block of at most 128 x 128 (Sec. 2, Eq. 1 applied to
 * the block alone): D <- D*, i.e. shortest paths that stay inside the block.
 * opts->closure picks the Eq. 1 k-loop or squaring to a fixpoint (Sec. 3.2).
 * n in [0, 128]; otherwise APSP_E_UNSUPPORTED.
 */
apsp_status_t apsp_closure(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                           void *D, int64_t ldd, const apsp_opts_t *opts, void *stream);

/*
 * All-pairs shortest paths by three-phase blocked Floyd-Warshall (Sec. 2,
 * Eq. 1): for each round of width b, close the diagonal tile, update its row
 * and column panels, then every remaining tile with one min-plus product.
 * D (n x n, ldd >= n) is overwritten with distances.  opts may be NULL.
 * By default round r+1's pivot closure and panel updates run on a second
 * stream of the context, overlapped with the rest of round r's remainder
 * update; with k-loop closures round r's update of pivot block r+1 and its
 * closure are one launch there (APSP_FLAG_NO_LOOKAHEAD keeps everything on
 * `stream`); the call still returns with all work ordered before later
 * work on `stream`.
 */
apsp_status_t apsp_fw(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                      void *D, int64_t ldd, const apsp_opts_t *opts, void *stream);

/*
 * All-pairs shortest paths by the R-Kleene recursion (Sec. 3.3, Eq. 4): split
 * D into [[A, B], [C, D]], close A, update B, C and D through A, close D,
 * update B and C through D and finally A.  Sub-blocks are strided views of
 * the one buffer; products whose output is also an operand run in place
 * (every stored value stays the length of a real walk, so the int32 result
 * is exact; fp32 results stay within rounding of the exact distances).
 */
apsp_status_t apsp_rkleene(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                           void *D, int64_t ldd, const apsp_opts_t *opts, void *stream);

/*
 * All-pairs shortest paths by repeated min-plus squaring (Sec. 3.2):
 * D <- min(D, D (min,+) D) until a pass changes nothing, at most
 * ceil(log2(n-1)) passes of change (by then every shortest path, of at most
 * n - 1 edges, is covered).  For n <= 2048 without APSP_FLAG_PACKED16 or
 * APSP_FLAG_SKIP_INF every pass runs inside one launch (tasks of a pass wait
 * on the previous pass's counter in the context scratch; no host
 * synchronisation); otherwise one launch per pass, and `stream` is
 * synchronised once per pass to read the device "changed" flag.  Passes
 * are in place (int32 exact; fp32 within rounding of the exact distances).
 * apsp_square_passes reports the number of passes of the last call.
 */
apsp_status_t apsp_square(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                          void *D, int64_t ldd, const apsp_opts_t *opts, void *stream);

/*
 * Passes the last apsp_square call on this context ran: a pass that changes
 * nothing ends the loop and is counted; the one-launch form also stops after
 * ceil(log2(n-1)) passes (0 for n <= 2).  After a one-launch call this
 * waits for `stream` (that call's stream) and reads the count from the
 * device.  APSP_E_STATE if apsp_square has not run on the context.
 */
apsp_status_t apsp_square_passes(apsp_ctx_t *ctx, void *stream, int32_t *h_passes);

/*
 * APSP_FLAG_PACKED16 (int32 only; other dtypes: APSP_E_UNSUPPORTED, and
 * minplus_gemm / apsp_closure / apsp_batched reject it).  The min-plus
 * products of apsp_fw / apsp_rkleene / apsp_square stage every value capped
 * at 14847 as a 16-bit pattern and fold four reduction steps with one 64-bit
 * add and one packed three-way minimum, half the instructions per term of
 * int32; the matrix in memory stays int32.  Capping commutes with min and +,
 * so an entry below the cap is exact.  After the solve one pass counts
 * entries >= 14847 and reads the count back (the call then returns with
 * `stream` synchronised); if there are any, the int32 solver runs once more
 * on the result, which yields the exact int32 closure.  The output is
 * therefore identical to the int32 solver's in every case; the mode pays
 * off when all distances are below 14847 and every vertex reaches every
 * other.
 * apsp_packed16_counts reports how many solves used the mode and how many
 * of them were redone.
 */
apsp_status_t apsp_packed16_counts(apsp_ctx_t *ctx, int64_t *runs, int64_t *redone);

/* Dispatches to apsp_fw / apsp_rkleene / apsp_square per opts->algo.  With
 * every option automatic (opts == NULL or all fields 0), a cost model whose
 * K equals apsp_candidate_count() loaded (apsp_costmodel_load / _set_params)
 * and a workspace of apsp_workspace_size(APSP_OP_SOLVE, n), the cost model
 * plans the solve from the matrix itself: one pass over D computes the four
 * features (as apsp_features), the inference kernel scores every candidate,
 * and the scores are read back (`stream` is synchronised once); the solve
 * then runs the best candidate the dtype can run.  Otherwise (or with any
 * option set) the size rule decides: blocked FW up to n = 4096, R-Kleene
 * with a 4096 FW cutover above, keeping the given options. */
apsp_status_t apsp_solve(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                         void *D, int64_t ldd, const apsp_opts_t *opts, void *stream);

/* Candidate index the last automatic apsp_solve on this context ran (-1 when
 * the size rule decided). */
apsp_status_t apsp_solve_choice(apsp_ctx_t *ctx, int32_t *h_choice);

/*
 * The cost model's four inputs for the n x n cost matrix D (see
 * apsp_costmodel_init): log2 n, log10 density with density = m / (n (n-1))
 * and m the finite off-diagonal entries (clamped to 1e-9), log2 of the batch
 * (0 here), and 1 when the graph is weakly connected (edges taken as
 * undirected; a lock-free union-find over the edges in the workspace) else
 * 0.  Synchronous: one pass over D, then the four floats are read back into
 * h_features.  Needs a workspace of apsp_workspace_size(APSP_OP_SOLVE, n)
 * bytes (APSP_E_NOMEM otherwise); with apsp_plan a C caller plans from a
 * matrix alone.
 */
apsp_status_t apsp_features(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n, const void *D, int64_t ldd,
                            void *stream, float *h_features);

/*
 * Last-hop predecessors (Sec. 2: pred[i][j] is the vertex before j on the
 * i -> j path, recovered by following pred back from j; Sec. 3.1 obtains it
 * with an argmin over the intermediate index).  From distances D (n x n,
 * ldd) and costs W (n x n, ldw) of the same dtype, writes the int32 matrix P
 * (n x n, ldp):
 *     P[i][j] = the smallest v != j minimising D[i][v] (+) W[v][j],
 *               -1 when i == j or that minimum is not below INF.
 * When D is the APSP result of W and every off-diagonal cost is positive
 * (the paper's assumption), P[i][j] is the last vertex before j on a shortest
 * i -> j path and following P from j reaches i.  P must not overlap D or W.
 * Same as apsp_predecessors_ex with APSP_PRED_AUTO.
 */
apsp_status_t apsp_predecessors(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                                const void *D, int64_t ldd, const void *W, int64_t ldw,
                                int32_t *P, int64_t ldp, void *stream);

/* Forms of the predecessor computation (all give the same P). */
#define APSP_PRED_AUTO   0  /* sparse when W has at most n^2/4 edges, they fit the workspace and
                               n <= 65535, else dense */
#define APSP_PRED_DENSE  1  /* one argmin product over every v: n^3 terms (add, compare, two selects) */
#define APSP_PRED_SPARSE 2  /* only the in-edges of j: n * m candidates; n <= 65535 */

/*
 * apsp_predecessors with a chosen form.  Only v with W[v][j] < INF can make
 * D[i][v] (+) W[v][j] fall below INF, so the sparse form takes the argmin
 * over j's in-edges alone: on the device it counts W's edges per row and
 * column range, scans the counts into an edge-list layout in the workspace,
 * lists the m edges and folds (value, v) keys with 64-bit LDS atomic minima,
 * ties to the smallest v.  Whether the sparse or the dense form writes P is
 * decided on the device (both are enqueued; the other returns at once):
 * sparse when the edge list fits the workspace and, for APSP_PRED_AUTO,
 * m <= n^2/4.  Nothing is read back, so every form only enqueues.  Without a
 * workspace larger than its fixed part (flag, counts, offsets), AUTO runs
 * the dense form and SPARSE returns APSP_E_NOMEM.  All forms give the same
 * P.  Errors: method outside 0..2 is APSP_E_ARG; APSP_PRED_SPARSE with
 * n > 65535 is APSP_E_UNSUPPORTED.
 */
apsp_status_t apsp_predecessors_ex(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                                   const void *D, int64_t ldd, const void *W, int64_t ldw,
                                   int32_t *P, int64_t ldp, int32_t method, void *stream);

/*
 * Path reconstruction (Sec. 2: the shortest path is recovered by following
 * the predecessor of the target back to the source).  For each of `count`
 * queries q, follows P (n x n int32, ldp, as written by apsp_predecessors)
 * back from d_dst[q] to d_src[q] and writes the path's vertices, source
 * first, to d_paths[q * max_len ...]; d_len[q] receives the number of
 * vertices: 1 when source == target, 0 when the target is unreachable
 * (P[s][t] < 0), -1 when a vertex index is out of range, the chain leaves
 * [0, n) or the path has more than min(max_len, n) vertices.  All arrays are
 * device memory (d_src, d_dst, d_len: count int32; d_paths: count * max_len
 * int32); one lane per query, enqueued only.  Errors: APSP_E_ARG for
 * count < 0, max_len < 1 or a NULL array.
 */
apsp_status_t apsp_path(apsp_ctx_t *ctx, int64_t n, const int32_t *P, int64_t ldp, int32_t count,
                        const int32_t *d_src, const int32_t *d_dst, int32_t *d_paths, int32_t max_len,
                        int32_t *d_len, void *stream);

/*
 * Many independent graphs, solved together.  `data` holds `count` square
 * row-major matrices back to back; d_offsets[g] (int64, device) is the
 * element offset of graph g and d_sizes[g] (int32, device) its n; h_sizes is
 * the same sizes on the host (used to plan, never dereferenced on device).
 * Every matrix is overwritten with its distances (Sec. 2, Eq. 1 per graph,
 * blocked into rounds).  n <= 1024 per graph for the lock-step and
 * persistent schedules, n <= 8192 for the queue schedule (APSP_E_UNSUPPORTED
 * beyond: use apsp_solve).
 *
 * Plan.  With every option automatic (opts NULL or all fields 0) the cost
 * model picks one of the batch candidates (apsp_batch_candidate) from the
 * batch's features (apsp_plan_batch; the density is counted on the device
 * and read back, so the first call with a new batch shape synchronises
 * `stream`); without a model with batch outputs the default candidate runs
 * (the queue schedule with 64 x 64 sub-tiles for n > 128).  A batch with a
 * graph above n = 1024 takes the best-scored queue candidate, and a batch of
 * fewer graphs than the device has XCDs takes it with
 * APSP_FLAG_BATCH_GLOBAL.  The plan is made once per batch shape
 * (apsp_batched_choice reports the candidate).  Otherwise the flags select
 * the schedule:
 *
 * APSP_FLAG_BATCH_QUEUE: a dependency-driven schedule in one launch: every
 * graph's first pivot closure, panel tiles, remainder tiles and next pivots
 * are tasks of one workgroup each, in one ticket queue per XCD (a graph's
 * tasks all run on one XCD, so its tiles are written and read through one
 * L2).  Each workgroup takes the next ticket of its XCD's queue when it
 * starts and waits, on per-graph counters in the plan memory, only for
 * tasks with smaller tickets, so every queue drains; waits are bounded
 * (apsp_batched_status reports an overrun).  The tickets follow a list
 * schedule simulated on the host (longest estimated path first).  Graphs
 * with n > opts->reserved[0] (all when 0) take round width opts->block
 * (64 or 128; 0 = 128) and, with opts->tile = APSP_TILE_64 and 128-wide
 * rounds, products cut into 64 x 64 sub-tile tasks; the others take 128-wide
 * rounds of whole tiles.  With APSP_FLAG_BATCH_GLOBAL all tasks share one
 * queue, so one graph's tasks spread over every XCD; a task then writes its
 * tile back beyond its XCD's L2 (an agent-scope release) before it signals.
 *
 * APSP_FLAG_BATCH_LOCKSTEP: all graphs advance one 128-wide round per launch
 * group -- the panel tiles of every graph, then the next round's pivot tiles
 * (updated and closed) on the context's second stream beside every other
 * remainder tile -- after one launch of all round-0 pivot closures; at most
 * 3 * ceil(max n / 128) launches; when every graph has n <= 128 the schedule
 * is the one closure launch, issued directly.
 *
 * APSP_FLAG_BATCH_PERSISTENT: one persistent kernel whose workgroups take
 * whole graphs, largest first, from an atomic queue.
 *
 * The queue, lock-step and persistent launches are captured once per batch
 * shape in a HIP graph and replayed (the buffers of each call are written to
 * a small device record first, so any buffers work);
 * APSP_FLAG_BATCH_NO_GRAPH launches directly; APSP_FLAG_BATCH_PER_GRAPH
 * issues one launch of the persistent kernel per graph (a baseline).  The
 * plan lives in the workspace (apsp_workspace_size with APSP_OP_BATCHED); a
 * workspace that is missing or too small is APSP_E_NOMEM, returned before
 * anything is enqueued.  A call with a new batch shape, or after another
 * call used the workspace, uploads the plan and synchronises `stream`; calls
 * on one context must not overlap across streams.
 */
apsp_status_t apsp_batched(apsp_ctx_t *ctx, apsp_dtype_t dtype, int32_t count,
                           void *data, const int64_t *d_offsets, const int32_t *d_sizes,
                           const int32_t *h_sizes, const apsp_opts_t *opts, void *stream);

/*
 * Diagnostic of the APSP_FLAG_BATCH_QUEUE schedule: *h_flags receives the
 * error word of the last batched plan (bit 0: a dependency wait overran its
 * bounded poll count; bit 1: a queue handed out fewer tickets than it holds,
 * i.e. some tasks did not run -- either means that launch's results are not
 * guaranteed) and the word is cleared.  Synchronises `stream`.  0 when no
 * batched plan is resident.
 */
apsp_status_t apsp_batched_status(apsp_ctx_t *ctx, void *stream, uint32_t *h_flags);

/*
 * apsp_batched for callers that cannot allocate device memory or register a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same schedules and results as apsp_batched,
 * with the plan held in a fixed 8 MiB device array of the library (one per
 * GPU, kept until the process ends; its address is resolved by apsp_create)
 * instead of the workspace.  Allocates and frees nothing; launches directly
 * (no graph replay).  A batch whose plan does not fit (about 500 k work
 * items: e.g. a few thousand graphs of n <= 512) is APSP_E_UNSUPPORTED,
 * returned before anything is enqueued.  Every call on one GPU shares that
 * array, which keeps the last call's plan: a call uploads its plan (and
 * synchronises `stream`) when the array holds another one, and calls that
 * overlap on one GPU -- from any context or thread -- race and must not be
 * made.
 */
apsp_status_t apsp_batched_noalloc(apsp_ctx_t *ctx, apsp_dtype_t dtype, int32_t count,
                                   void *data, const int64_t *d_offsets, const int32_t *d_sizes,
                                   const int32_t *h_sizes, const apsp_opts_t *opts, void *stream);

/*
 * Checks the input contract of an n x n matrix (Sec. 3.1 and 3.4): diagonal
 * exactly 0; int32 entries in [0, INF]; fp32 entries >= 0 and not NaN.
 * Synchronous: waits for `stream`, writes the number of violating entries to
 * *h_violations and returns APSP_E_INPUT if it is non-zero.
 */
apsp_status_t apsp_validate(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n,
                            const void *D, int64_t ldd, void *stream, int64_t *h_violations);

/*
 * Candidate plans.  A fixed table of (algorithm, round width / leaf size,
 * tile, closure, cutover, flags) choices indexed 0..apsp_candidate_count()-1;
 * the autotuner times every one of them and the cost model scores them.
 * Some carry APSP_FLAG_PACKED16 (int32 data only).
 */
int32_t apsp_candidate_count(void);
apsp_status_t apsp_candidate(int32_t index, apsp_opts_t *out);

/*
 * Cost model: a small MLP, 4 features -> 64 -> 64 -> K (ReLU hidden layers),
 * whose K outputs are predicted normalised log run times of the K candidate
 * plans; the plan is the argmin.  Features of one graph, in this order:
 *   log2(n), log10(density) with density = edges / (n (n-1)) (clamped to
 *   1e-9), 0 (log2 of a batch of one), 1 if the graph is weakly connected
 *   else 0; of a batch: see apsp_plan_batch.  A model that plans both has
 *   apsp_candidate_count() + apsp_batch_candidate_count() outputs, the
 *   single-graph candidates first.
 * Parameters are one fp32 array, row-major input x output:
 *   W1[4][64] | b1[64] | W2[64][64] | b2[64] | W3[64][K] | b3[K]
 * (4480 + 65 K floats).  Inputs are standardised inside the kernels with the
 * stored mean/deviation.  Training is full-batch masked mean squared error
 * with Adam, run entirely inside one kernel launch; every reduction has a
 * fixed order, so results are deterministic.  Device pointers (d_*) are
 * caller-owned; rows <= 4096.  The context owns the parameters, the Adam
 * moments and a small activation workspace, allocated by apsp_costmodel_init.
 */
typedef struct apsp_train_cfg {
    int32_t steps;     /* Adam steps in this call (>= 1) */
    float lr, beta1, beta2, eps;
    int32_t reserved[3];
} apsp_train_cfg_t;

/* (Re)initialises a K-output model with He-uniform weights from a
 * counter-based hash of `seed`, zero biases, zero Adam state, identity
 * standardisation.  K must equal apsp_candidate_count() for apsp_plan. */
apsp_status_t apsp_costmodel_init(apsp_ctx_t *ctx, int32_t K, uint64_t seed);
apsp_status_t apsp_costmodel_set_norm(apsp_ctx_t *ctx, const float *h_mu4, const float *h_sd4);
/* Copies count = 4480 + 65 K floats in / out (host memory); set resets Adam. */
apsp_status_t apsp_costmodel_set_params(apsp_ctx_t *ctx, const float *h_params, int64_t count);
apsp_status_t apsp_costmodel_get_params(apsp_ctx_t *ctx, float *h_params, int64_t count);
/* Model file I/O (plain text, so a trained model moves between processes
 * and languages): "apsp-costmodel 1", then K, the layer sizes, the four
 * feature means and deviations and the 4480 + 65 K parameters, every value
 * printed with 9 significant digits (binary32 reads back exactly).  Save
 * waits for the device and needs a model; load parses and checks the whole
 * file (header, sizes equal to this library's, finite values, deviations
 * > 0) before it changes the context, then initialises a model of that K if
 * needed and sets the standardisation and parameters (Adam state reset).
 * APSP_E_ARG for a NULL path, a file that cannot be opened or written, or a
 * malformed file (the context is then unchanged). */
apsp_status_t apsp_costmodel_save(apsp_ctx_t *ctx, const char *path);
apsp_status_t apsp_costmodel_load(apsp_ctx_t *ctx, const char *path);
/* d_X rows x 4, d_T and d_mask rows x K (mask 1 = target present).  d_losses
 * (steps floats, may be NULL) receives the loss before each step. */
apsp_status_t apsp_costmodel_train(apsp_ctx_t *ctx, const float *d_X, const float *d_T, const float *d_mask,
                                   int32_t rows, const apsp_train_cfg_t *cfg, float *d_losses, void *stream);
/* Gradient of the loss at the current parameters (no update) into d_grad
 * (4480 + 65 K floats) and the loss into *d_loss (may be NULL). */
apsp_status_t apsp_costmodel_grad(apsp_ctx_t *ctx, const float *d_X, const float *d_T, const float *d_mask,
                                  int32_t rows, float *d_grad, float *d_loss, void *stream);
/* d_out rows x K predictions. */
apsp_status_t apsp_costmodel_forward(apsp_ctx_t *ctx, const float *d_X, int32_t rows, float *d_out, void *stream);
/* d_choice rows int32: argmin candidate per row (first minimum). */
apsp_status_t apsp_costmodel_predict(apsp_ctx_t *ctx, const float *d_X, int32_t rows, int32_t *d_choice,
                                     void *stream);

/* Plan for one graph of `dtype` (synchronous; batch must be 1): the cost
 * model's argmin over the candidates that dtype can run (fp32 skips the
 * APSP_FLAG_PACKED16 ones) when a model with at least apsp_candidate_count()
 * outputs is loaded, else a size rule (blocked FW up to n = 4096, R-Kleene
 * with a 4096 FW cutover above).  *h_choice (may be NULL) gets the candidate
 * index, or -1 for the size rule. */
apsp_status_t apsp_plan(apsp_ctx_t *ctx, apsp_dtype_t dtype, int64_t n, double density, int32_t batch,
                        int32_t connected, apsp_opts_t *out, int32_t *h_choice);

/*
 * Batch candidate plans of apsp_batched (schedule flags, round width, tile,
 * reserved[0] = the n above which a graph takes that width and tile), indexed
 * 0 .. apsp_batch_candidate_count() - 1: lock-step; queue with whole
 * 128-tiles; queue with 64 x 64 sub-tiles for n > 128; for n > 256; queue
 * with 64-wide rounds for n > 384; persistent.
 */
int32_t apsp_batch_candidate_count(void);
apsp_status_t apsp_batch_candidate(int32_t index, apsp_opts_t *out);

/*
 * Plan for a batch (synchronous): when the loaded model has
 * apsp_candidate_count() + apsp_batch_candidate_count() outputs (the batch
 * candidates last), the argmin of its batch outputs for the features
 * log2(largest n), log10(density) with density = edges / sum n (n-1) over
 * the batch (clamped to 1e-9), log2(count), and the share of the batch's
 * work (sum of n^3) in graphs with n > 256; else the default candidate.
 * *h_choice (may be NULL) gets the batch candidate index, or -1 for the
 * default.
 */
apsp_status_t apsp_plan_batch(apsp_ctx_t *ctx, apsp_dtype_t dtype, int32_t count, const int32_t *h_sizes,
                              double density, apsp_opts_t *out, int32_t *h_choice);

/* Batch candidate the last automatic apsp_batched plan chose (-1: none yet). */
apsp_status_t apsp_batched_choice(apsp_ctx_t *ctx, int32_t *h_choice);

/*
 * Kernel timing for measurement tools (not needed to compute anything).
 * While enabled, every kernel the context launches is bracketed by two HIP
 * events recorded on the launch stream; apsp_profile_read synchronises those
 * events and returns, per kernel kind, the number of launches, their summed
 * duration and their summed algorithmic work.  A min-plus term is one
 * (a + b) followed by one min.  Enabling clears previous records.
 */
#define APSP_KERNEL_MINPLUS_128 0   /* min-plus product, 128 x 128 tiles */
#define APSP_KERNEL_MINPLUS_64  1   /* min-plus product, 64 x 64 tiles */
#define APSP_KERNEL_CLOSURE     2   /* diagonal-tile closure */
#define APSP_KERNEL_OTHER       3   /* validation, fills, batched, cost model */
#define APSP_KERNEL_KINDS       4

typedef struct apsp_kernel_stats {
    int64_t launches;
    double  milliseconds;   /* sum of event-timed launch durations */
    double  terms;          /* sum of min-plus terms (M*N*K per product; s^3 per k-loop closure) */
    double  bytes;          /* sum of compulsory HBM bytes: operands read once, C read and written once */
} apsp_kernel_stats_t;

/* on = 0 stops recording, 1 records every kind, any other value is a bit
 * mask (1 << APSP_KERNEL_*) of the kinds to record -- recording only the
 * kernel under study keeps the events from perturbing the others. */
apsp_status_t apsp_profile_enable(apsp_ctx_t *ctx, int32_t on);
apsp_status_t apsp_profile_read(apsp_ctx_t *ctx, int32_t kind, apsp_kernel_stats_t *out);

/*
 * Issue-rate calibration for measurement tools (Sec. 3, Eq. 2: the fold is
 * the product's inner step).  Runs a spin kernel over the whole device in
 * which every lane repeats the fold's own instructions on registers, with
 * independent chains so nothing waits: APSP_FOLD_I32 (one 64-bit add for two
 * sums, one v_min3_u32), APSP_FOLD_F32 (two v_add_f32, one v_min3_f32),
 * APSP_FOLD_PACKED16 (one 64-bit add for four 16-bit sums, one
 * v_pk_minimum3_f16).  Synchronous on `stream` (a warm-up launch, then one
 * event-timed launch of roughly 10-20 ms); writes the achieved min-plus
 * terms/s and VALU lane-instructions/s -- the ceiling the product kernels
 * can reach at the clock the device runs now.  Touches one word of the
 * context's scratch.  APSP_E_ARG for an unknown fold or NULL outputs.
 */
#define APSP_FOLD_I32      0
#define APSP_FOLD_F32      1
#define APSP_FOLD_PACKED16 2
apsp_status_t apsp_measure_fold_rate(apsp_ctx_t *ctx, int32_t fold, void *stream, double *h_terms_per_s,
                                     double *h_lane_instr_per_s);

#ifdef __cplusplus
}
#endif

#endif /* APSP_H */
