// C ABI of libapsp (include/apsp.h) and the host drivers that sequence the
// kernels: the blocked Floyd-Warshall round loop, the R-Kleene recursion and
// min-plus squaring.  Every driver only enqueues work on the caller's
// stream; argument checks run before the first HIP call.
#include "apsp.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <utility>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

// Fixed device scratch of apsp_batched_noalloc, for callers that cannot
// allocate: each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes this name to a kernel or a copy (in
// host code it is a stand-in, not a device address): apsp_create resolves
// the device address once per GPU (hipGetSymbolAddress) and every use goes
// through that address.  Word 0 is the persistent queue's ticket counter;
// the batch plan starts at byte 256.
constexpr size_t kFixedScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double terms, bytes;
};

struct apsp_ctx {
    int device = 0;
    int num_cus = 256;
    void* d_scratch = nullptr;      // counters and flags (allocated by apsp_create)
    size_t scratch_bytes = 0;
    char* ws = nullptr;             // caller's workspace (apsp_set_workspace)
    size_t ws_bytes = 0;
    int ws_owner = 0;               // what the workspace holds now (WS_*)
    char* fixed = nullptr;          // device address of this GPU's fixed scratch
    uint64_t fixed_serial = 0;      // upload serial of this context's plan in it (0: none)
    hipStream_t capture = nullptr;  // private stream used only for graph capture
    hipStream_t side = nullptr;     // second stream of the FW look-ahead
    hipEvent_t ev_a = nullptr;      // look-ahead: band r+1 current
    hipEvent_t ev_p = nullptr;      // look-ahead: pivot r+1 and panels done
    hipEvent_t ev_b = nullptr;      // look-ahead: the previous round's remainder done
    // cached batched plan: queue order on the device and the captured launch
    uint64_t bkey = 0;
    int32_t bcount = 0;
    int32_t bdtype = -1;
    std::vector<int32_t> border;
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    hipGraphNode_t bnode = nullptr;
    hipKernelNodeParams bparams{};
    apsp::BatchArgs bargs{};
    // lock-step batched schedule: work items and launch list, captured graph
    std::vector<int4> litems;
    struct Launch { int phase, offset, count; bool side; };   // side: on the second stream
    std::vector<Launch> llaunches;
    uint64_t graph_key = 0;         // plan key the captured graphs were made for
    uint32_t* batch_err = nullptr;  // error word of the queue schedule's last plan memory
    hipGraph_t lgraph = nullptr;
    hipGraphExec_t lexec = nullptr;
    // dependency-driven batched schedule: tasks, counter count, captured graph
    std::vector<apsp::BatchTask> qtasks;
    std::vector<int32_t> qoff;      // queue x: tasks qoff[x] .. qoff[x+1] (one queue per XCD)
    int32_t qcounters = 0;
    hipGraph_t qgraph = nullptr;
    hipGraphExec_t qexec = nullptr;
    // cost model
    int32_t cm_K = 0;
    float* cm_params = nullptr;     // device: parameters, Adam moments, gradients
    float* cm_m = nullptr;
    float* cm_v = nullptr;
    float* cm_grad = nullptr;
    float* cm_ws = nullptr;         // activation workspace for kCmMaxRows rows
    float* cm_io = nullptr;         // plan: 4 features, K outputs, 1 choice
    float* h_io = nullptr;          // pinned host copy of the plan read-back (4 KB)
    int32_t square_passes = -1;     // passes of the last apsp_square (host-driven form)
    bool square_passes_device = false;   // ... or in the scratch (one-launch form)
    int32_t cm_steps = 0;           // Adam steps taken since init / set_params
    apsp::MlpNorm cm_norm{};
    bool prof = false;              // kernel timing enabled
    uint32_t prof_mask = 0;         // bit k set: record kernels of kind k
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    int32_t last_choice = -1;       // candidate apsp_solve(auto) ran last (-1: size rule)
    uint64_t bauto_key = 0;         // batch shape the automatic batched plan was made for
    int32_t bauto_choice = -1;      // its batch candidate
    int64_t p16_runs = 0;           // solves run with APSP_FLAG_PACKED16
    int64_t p16_redone = 0;         // ... of which were redone in int32
    uint32_t magic = 0x41505350;    // "APSP"
};

namespace {

thread_local std::string g_last_error;

apsp_status_t fail(apsp_status_t st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

apsp_status_t hip_fail(hipError_t e, const char* where)
{
    return fail(APSP_E_HIP, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(expr, where)                         \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// Forced failure for host-side error-path tests: APSP_FAULT=launch makes the
// first kernel enqueue of a call report a HIP error without touching a GPU.
bool fault_injected(const char* what)
{
    const char* f = getenv("APSP_FAULT");
    return f && strcmp(f, what) == 0;
}

apsp_status_t check_ctx(apsp_ctx_t* ctx)
{
    if (!ctx) return fail(APSP_E_ARG, "context is NULL");
    if (ctx->magic != 0x41505350) return fail(APSP_E_STATE, "context is not valid (destroyed?)");
    return APSP_OK;
}

apsp_status_t check_dtype(apsp_dtype_t dt)
{
    if (dt != APSP_I32 && dt != APSP_F32) return fail(APSP_E_ARG, "unknown dtype %d", (int)dt);
    return APSP_OK;
}

apsp_status_t check_square(int64_t n, const void* D, int64_t ld)
{
    if (n < 0) return fail(APSP_E_ARG, "n = %lld is negative", (long long)n);
    if (n > (int64_t)1 << 30) return fail(APSP_E_ARG, "n = %lld is too large", (long long)n);
    if (n > 0 && !D) return fail(APSP_E_ARG, "matrix pointer is NULL");
    if (n > 0 && ld < n) return fail(APSP_E_ARG, "ld = %lld < n = %lld", (long long)ld, (long long)n);
    return APSP_OK;
}

// ---------------------------------------------------------------------------
// optional kernel timing: events recorded on the launch stream around a launch
// ---------------------------------------------------------------------------
hipEvent_t take_event(apsp_ctx_t* ctx)
{
    if (ctx->pool_used == ctx->pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->pool.push_back(e);
    }
    return ctx->pool[ctx->pool_used++];
}

template <class F>
apsp_status_t timed(apsp_ctx_t* ctx, int kind, double terms, double bytes, hipStream_t st, F&& launch)
{
    if (!ctx->prof || !(ctx->prof_mask & (1u << kind))) return launch();
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return launch();
    hipEventRecord(a, st);
    apsp_status_t rc = launch();
    hipEventRecord(b, st);
    ctx->recs.push_back({kind, a, b, terms, bytes});
    return rc;
}

void group_work(const apsp::GemmGroup& g, int tile, double& terms, double& bytes)
{
    const apsp::TileShape ts = apsp::tile_shape(tile);
    terms = bytes = 0;
    for (int i = 0; i < g.count; ++i) {
        const apsp::GemmProblem& p = g.p[i];
        auto excluded = [](int64_t total, int64_t t0, int64_t tc, int64_t w) {
            if (!tc) return (int64_t)0;
            return std::min(total, (t0 + tc) * w) - std::min(total, t0 * w);
        };
        const double m = (double)(p.M - excluded(p.M, p.skip_m0, p.skip_mc, ts.mt));
        const double n = (double)(p.N - excluded(p.N, p.skip_n0, p.skip_nc, ts.nt));
        terms += m * n * (double)p.K;
        bytes += 4.0 * (m * p.K + (double)p.K * n + 2.0 * m * n);
    }
}

const apsp_opts_t* opts_or_default(const apsp_opts_t* o)
{
    static const apsp_opts_t zero{};
    return o ? o : &zero;
}

apsp_status_t check_opts(const apsp_opts_t* o)
{
    if (o->block != 0 && o->block != 64 && o->block != 128)
        return fail(APSP_E_ARG, "block = %d (allowed: 0, 64, 128)", o->block);
    if (o->tile < 0 || o->tile > APSP_TILE_64) return fail(APSP_E_ARG, "tile = %d", o->tile);
    if (o->closure < 0 || o->closure > APSP_CLOSURE_SQUARE) return fail(APSP_E_ARG, "closure = %d", o->closure);
    if (o->algo < 0 || o->algo > APSP_ALGO_SQUARE) return fail(APSP_E_ARG, "algo = %d", o->algo);
    if (o->cutover < 0) return fail(APSP_E_ARG, "cutover = %d", o->cutover);
    return APSP_OK;
}

size_t esize(apsp_dtype_t) { return 4; }

char* elem(void* base, apsp_dtype_t dt, int64_t r, int64_t c, int64_t ld)
{
    return static_cast<char*>(base) + (r * ld + c) * (int64_t)esize(dt);
}

struct Plan {
    int block;      // FW round width / R-Kleene leaf size
    int tile;       // GEMM tile (APSP_TILE_AUTO: chosen per product)
    int closure;    // 1 k-loop, 2 squaring
    int cutover;    // R-Kleene -> FW below this size
    bool splitk;
    bool lookahead; // FW: overlap the next pivot and panels with the remainder
    bool p16;       // int32: min-plus products in capped 16-bit arithmetic
    bool skip;      // products skip reduction slices with an all-INF operand
    bool det;       // aliased product operands are read from a copy (tmp)
    void* tmp = nullptr;   // workspace for those copies (det)
};

Plan resolve(const apsp_opts_t* o)
{
    Plan p;
    p.block = o->block ? o->block : 128;
    p.tile = o->tile;   // APSP_TILE_AUTO (0) lets pick_tile decide per product
    p.closure = o->closure ? o->closure : APSP_CLOSURE_KLOOP;
    p.cutover = o->cutover;
    p.splitk = !(o->flags & APSP_FLAG_NO_SPLITK);
    p.lookahead = !(o->flags & APSP_FLAG_NO_LOOKAHEAD);
    p.p16 = (o->flags & APSP_FLAG_PACKED16) != 0;
    p.det = (o->flags & APSP_FLAG_DETERMINISTIC) != 0;
    p.skip = (o->flags & APSP_FLAG_SKIP_INF) != 0;
    return p;
}

// element semantics of the min-plus products of a plan
apsp::DType gemm_dtype(apsp_dtype_t dt, const Plan& pl)
{
    return pl.p16 ? apsp::I32P16 : (apsp::DType)dt;
}

apsp::GemmProblem make_problem(apsp_dtype_t dt, void* base, int64_t ld,
                               int64_t ar, int64_t ac,      // A origin
                               int64_t br, int64_t bc,      // B origin
                               int64_t cr, int64_t cc,      // C origin
                               int64_t M, int64_t N, int64_t K)
{
    apsp::GemmProblem p{};
    p.A = elem(base, dt, ar, ac, ld);
    p.B = elem(base, dt, br, bc, ld);
    p.C = elem(base, dt, cr, cc, ld);
    p.lda = p.ldb = p.ldc = ld;
    p.M = (int32_t)M;
    p.N = (int32_t)N;
    p.K = (int32_t)K;
    return p;
}

// Tile for a product: small outputs use 64 x 64 tiles to fill the device.
int pick_tile(const Plan& pl, int64_t M, int64_t N)
{
    if (pl.tile == apsp::TILE_64) return apsp::TILE_64;
    if (pl.tile == apsp::TILE_128) return apsp::TILE_128;
    // 128 x 128 tiles (with a split reduction below 512 tiles) from about
    // 2048 x 2048 up; 64 x 64 tiles fill the device better below that
    const int64_t t128 = ((M + 127) / 128) * ((N + 127) / 128);
    if (t128 < 256) return apsp::TILE_64;
    return apsp::TILE_128;
}

apsp_status_t run_group(apsp_ctx_t* ctx, apsp_dtype_t dt, apsp::GemmGroup& g, const Plan& pl,
                        int tile, hipStream_t st)
{
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    const apsp::DType gdt = gemm_dtype(dt, pl);
    apsp::finalize_group(g, tile, pl.splitk ? 2 * ctx->num_cus : 0, gdt);
    double terms, bytes;
    group_work(g, tile, terms, bytes);
    const int kind = tile == apsp::TILE_64 ? APSP_KERNEL_MINPLUS_64 : APSP_KERNEL_MINPLUS_128;
    return timed(ctx, kind, terms, bytes, st, [&]() -> apsp_status_t {
        HIP_TRY(apsp::launch_minplus(gdt, tile, g, pl.skip, st), "min-plus launch");
        return APSP_OK;
    });
}

apsp_status_t run_one(apsp_ctx_t* ctx, apsp_dtype_t dt, const apsp::GemmProblem& p, const Plan& pl,
                      hipStream_t st)
{
    if (p.M <= 0 || p.N <= 0 || p.K <= 0) return APSP_OK;
    apsp::GemmGroup g{};
    g.count = 1;
    g.p[0] = p;
    return run_group(ctx, dt, g, pl, pick_tile(pl, p.M, p.N), st);
}

apsp_status_t run_two(apsp_ctx_t* ctx, apsp_dtype_t dt, const apsp::GemmProblem& p,
                      const apsp::GemmProblem& q, const Plan& pl, hipStream_t st)
{
    apsp::GemmGroup g{};
    const int64_t mm = std::max<int64_t>(p.M, q.M), nn = std::max<int64_t>(p.N, q.N);
    if (p.M > 0 && p.N > 0 && p.K > 0) g.p[g.count++] = p;
    if (q.M > 0 && q.N > 0 && q.K > 0) g.p[g.count++] = q;
    if (!g.count) return APSP_OK;
    return run_group(ctx, dt, g, pl, pick_tile(pl, mm, nn), st);
}

apsp_status_t closure(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t s,
                      int kind, hipStream_t st)
{
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    const double terms = (double)s * s * s, bytes = 8.0 * s * s;
    return timed(ctx, APSP_KERNEL_CLOSURE, terms, bytes, st, [&]() -> apsp_status_t {
        HIP_TRY(apsp::launch_closure((apsp::DType)dt, kind, elem(D, dt, off, off, ld), ld, (int32_t)s, st),
                "closure launch");
        return APSP_OK;
    });
}

// ---------------------------------------------------------------------------
// Blocked Floyd-Warshall on the window [off, off+n) x [off, off+n)
// ---------------------------------------------------------------------------
// phases 1 and 2 of round (k0, bk): close the pivot tile, then the row panel
// R_KJ <- X* (min,+) R_KJ and the column panel C_IK <- C_IK (min,+) X*
// rows x cols block at (r, c) of D (stride ld) into dst (stride dld), on st
apsp_status_t copy_block(apsp_dtype_t dt, void* dst, int64_t dld, const void* D, int64_t ld, int64_t r, int64_t c,
                         int64_t rows, int64_t cols, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return APSP_OK;
    const size_t e = esize(dt);
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)dld * e, elem(const_cast<void*>(D), dt, r, c, ld), (size_t)ld * e,
                             (size_t)cols * e, (size_t)rows, hipMemcpyDeviceToDevice, st),
            "operand copy");
    return APSP_OK;
}

apsp_status_t fw_panels(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t n,
                        int64_t k0, int64_t bk, const Plan& pl, hipStream_t st)
{
    if (bk == n) return APSP_OK;
    const int t_p2 = apsp::TILE_64;                 // panels are thin: small tiles
    const apsp::TileShape s2 = apsp::tile_shape(t_p2);
    apsp::GemmGroup g2{};
    g2.count = 2;
    g2.p[0] = make_problem(dt, D, ld, off + k0, off + k0, off + k0, off, off + k0, off, bk, n, bk);
    g2.p[0].skip_n0 = (int32_t)(k0 / s2.nt);
    g2.p[0].skip_nc = (int32_t)((bk + s2.nt - 1) / s2.nt);
    g2.p[1] = make_problem(dt, D, ld, off, off + k0, off + k0, off + k0, off, off + k0, n, bk, bk);
    g2.p[1].skip_m0 = (int32_t)(k0 / s2.mt);
    g2.p[1].skip_mc = (int32_t)((bk + s2.mt - 1) / s2.mt);
    if (pl.det) {
        // the row panel (bk x n) and the column panel (n x bk) are read from
        // copies: a 64-tile of the band would otherwise read the band's other
        // tile rows (columns) while their workgroups lower them
        char* rowc = static_cast<char*>(pl.tmp);
        char* colc = rowc + (size_t)bk * n * esize(dt);
        apsp_status_t rc;
        if ((rc = copy_block(dt, rowc, n, D, ld, off + k0, off, bk, n, st)) ||
            (rc = copy_block(dt, colc, bk, D, ld, off, off + k0, n, bk, st)))
            return rc;
        g2.p[0].B = rowc;
        g2.p[0].ldb = n;
        g2.p[1].A = colc;
        g2.p[1].lda = bk;
    }
    return run_group(ctx, dt, g2, pl, t_p2, st);
}

apsp_status_t fw_pivot_panels(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t n,
                              int64_t k0, int64_t bk, const Plan& pl, hipStream_t st)
{
    apsp_status_t rc = closure(ctx, dt, D, ld, off + k0, bk, pl.closure, st);
    if (rc) return rc;
    return fw_panels(ctx, dt, D, ld, off, n, k0, bk, pl, st);
}

// Pivot block (k1, k1) of the next round, fused: round (k0, bk)'s update of
// that block from its panel blocks C(k1, k0) and R(k0, k1), then its closure.
apsp_status_t fw_pivot_fused(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t k0,
                             int64_t bk, int64_t k1, int64_t bk1, hipStream_t st)
{
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    const double terms = (double)bk1 * bk1 * (bk1 + bk), bytes = 8.0 * bk1 * bk1 + 8.0 * bk1 * bk;
    return timed(ctx, APSP_KERNEL_CLOSURE, terms, bytes, st, [&]() -> apsp_status_t {
        HIP_TRY(apsp::launch_pivot_fused(dt == APSP_F32 ? apsp::F32 : apsp::I32, elem(D, dt, off + k1, off + k1, ld),
                                         ld, elem(D, dt, off + k1, off + k0, ld), elem(D, dt, off + k0, off + k1, ld),
                                         (int32_t)bk1, (int32_t)bk, st),
                "fused pivot launch");
        return APSP_OK;
    });
}

// Remainder update D_IJ <- min(D_IJ, C_IK (min,+) R_KJ) of round (k0, bk) for
// the tiles whose row and column both lie outside the band [x0, x0 + xw)
// (x0 tile-aligned; the band covers the pivot band and possibly the next one).
apsp::GemmProblem remainder(apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t n, int64_t k0, int64_t bk,
                            int64_t x0, int64_t xw, const apsp::TileShape& ts)
{
    apsp::GemmProblem p = make_problem(dt, D, ld, off, off + k0, off + k0, off, off, off, n, n, bk);
    p.skip_m0 = (int32_t)(x0 / ts.mt);
    p.skip_mc = (int32_t)((xw + ts.mt - 1) / ts.mt);
    p.skip_n0 = (int32_t)(x0 / ts.nt);
    p.skip_nc = (int32_t)((xw + ts.nt - 1) / ts.nt);
    return p;
}

// ---------------------------------------------------------------------------
// Blocked Floyd-Warshall on the window [off, off+n) x [off, off+n)
//
// Sequential order per round: pivot closure, panels, remainder.  With
// look-ahead (default) the remainder of round r is split: first the tiles
// of band r+1 (its row and its column), then -- on the caller's stream -- all
// other tiles, while a second stream closes pivot r+1 and updates its panels
// as soon as band r+1 is current.  The second stream touches only band r+1,
// which the rest of round r neither reads nor writes; two events order the
// streams.  The latency-bound closure and thin panel products then run under
// the bulk remainder product instead of between rounds.
// ---------------------------------------------------------------------------
apsp_status_t fw_window(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t n,
                        const Plan& pl, hipStream_t st)
{
    const int64_t b = pl.block;
    // the excluded bands must be whole tiles: 64-wide rounds use 64-tiles.
    // The remainder's reduction is only one round wide, so a launch of
    // 128-tiles ends in a long partial wave that keeps the second stream's
    // panel products waiting for CUs; 64-tiles free slots sooner.  Measured
    // (int32, p = 0.02): n = 3072 3.25 -> 2.38 ms, 4096 3.76 -> 3.40, 6144
    // 10.1 -> 9.8, 8192 +2%; with capped 16-bit products 64-tiles also win
    // at 8192 (18.9 -> 16.6 ms).
    const int64_t rem64_max = pl.p16 ? 8192 : 6144;
    const int t_p3 = (b < 128 || (pl.tile == APSP_TILE_AUTO && n <= rem64_max)) ? (int)apsp::TILE_64
                                                                                 : pick_tile(pl, n, n);
    const apsp::TileShape s3 = apsp::tile_shape(t_p3), s64 = apsp::tile_shape(apsp::TILE_64);
    const int64_t rounds = (n + b - 1) / b;
    const bool ahead = pl.lookahead && rounds >= 3 && ctx->side && ctx->ev_a && ctx->ev_p;
    // with k-loop closures the next pivot is updated and closed by one fused
    // launch on the second stream from the start of each round
    const bool fused = ahead && pl.closure == APSP_CLOSURE_KLOOP && ctx->ev_b && b <= 128;
    apsp_status_t rc = fw_pivot_panels(ctx, dt, D, ld, off, n, 0, std::min(b, n), pl, st);
    if (rc) return rc;
    if (fused) HIP_TRY(hipEventRecord(ctx->ev_b, st), "look-ahead event");
    for (int64_t r = 0; r < rounds; ++r) {
        const int64_t k0 = r * b, bk = std::min(b, n - k0);
        if (bk == n) break;
        if (!ahead || r + 1 == rounds) {
            if (r > 0 && !ahead) {
                rc = fw_pivot_panels(ctx, dt, D, ld, off, n, k0, bk, pl, st);
                if (rc) return rc;
            }
            apsp::GemmGroup g3{};
            g3.count = 1;
            g3.p[0] = remainder(dt, D, ld, off, n, k0, bk, k0, bk, s3);
            rc = run_group(ctx, dt, g3, pl, t_p3, st);
            if (rc) return rc;
            continue;
        }
        const int64_t k1 = k0 + b, bk1 = std::min(b, n - k1);
        if (fused) {
            // (o) second stream, once the previous round's remainder is in:
            //     pivot r+1 updated from round r's panels, then closed
            HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->ev_b, 0), "look-ahead wait");
            rc = fw_pivot_fused(ctx, dt, D, ld, off, k0, bk, k1, bk1, ctx->side);
            if (rc) return rc;
        }
        // (a) band r+1: its row (all columns outside band r, and outside band
        //     r+1 when the pivot is fused) and its column (rows outside bands
        //     r and r+1), thin products on 64-tiles
        apsp::GemmGroup ga{};
        ga.count = 2;
        ga.p[0] = make_problem(dt, D, ld, off + k1, off + k0, off + k0, off, off + k1, off, bk1, n, bk);
        ga.p[0].skip_n0 = (int32_t)(k0 / s64.nt);
        ga.p[0].skip_nc = (int32_t)(((fused ? bk + bk1 : bk) + s64.nt - 1) / s64.nt);
        ga.p[1] = make_problem(dt, D, ld, off, off + k0, off + k0, off + k1, off, off + k1, n, bk1, bk);
        ga.p[1].skip_m0 = (int32_t)(k0 / s64.mt);
        ga.p[1].skip_mc = (int32_t)((bk + bk1 + s64.mt - 1) / s64.mt);
        rc = run_group(ctx, dt, ga, pl, apsp::TILE_64, st);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ctx->ev_a, st), "look-ahead event");
        // (b) second stream: pivot r+1 (unless fused) and its panels
        HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->ev_a, 0), "look-ahead wait");
        rc = fused ? fw_panels(ctx, dt, D, ld, off, n, k1, bk1, pl, ctx->side)
                   : fw_pivot_panels(ctx, dt, D, ld, off, n, k1, bk1, pl, ctx->side);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ctx->ev_p, ctx->side), "look-ahead event");
        // (c) caller's stream: every tile outside bands r and r+1
        apsp::GemmGroup gb{};
        gb.count = 1;
        gb.p[0] = remainder(dt, D, ld, off, n, k0, bk, k0, bk + bk1, s3);
        if (gb.p[0].M > 0) {
            rc = run_group(ctx, dt, gb, pl, t_p3, st);
            if (rc) return rc;
        }
        if (fused) HIP_TRY(hipEventRecord(ctx->ev_b, st), "look-ahead event");
        HIP_TRY(hipStreamWaitEvent(st, ctx->ev_p, 0), "look-ahead join");
    }
    return APSP_OK;
}

// ---------------------------------------------------------------------------
// R-Kleene on the window [off, off+n)^2 (Sec. 3.3, Eq. 4)
// ---------------------------------------------------------------------------
// Deterministic mode: the B block (rows a.., columns d.., n1 x n2) and the C
// block (rows d.., columns a.., n2 x n1) are copied to the workspace and the
// products that update them read the copy in place of the block itself
// (as operand B when b_is_B, else as operand A; likewise for C).
apsp_status_t aliased_from_copies(apsp_dtype_t dt, void* D, int64_t ld, int64_t a, int64_t d, int64_t n1,
                                  int64_t n2, const Plan& pl, apsp::GemmProblem& pb, bool b_is_B,
                                  apsp::GemmProblem& pc, bool c_is_B, hipStream_t st)
{
    char* bcopy = static_cast<char*>(pl.tmp);
    char* ccopy = bcopy + (size_t)n1 * n2 * esize(dt);
    apsp_status_t rc;
    if ((rc = copy_block(dt, bcopy, n2, D, ld, a, d, n1, n2, st)) ||
        (rc = copy_block(dt, ccopy, n1, D, ld, d, a, n2, n1, st)))
        return rc;
    if (b_is_B) {
        pb.B = bcopy;
        pb.ldb = n2;
    } else {
        pb.A = bcopy;
        pb.lda = n2;
    }
    if (c_is_B) {
        pc.B = ccopy;
        pc.ldb = n1;
    } else {
        pc.A = ccopy;
        pc.lda = n1;
    }
    return APSP_OK;
}

apsp_status_t rk_window(apsp_ctx_t* ctx, apsp_dtype_t dt, void* D, int64_t ld, int64_t off, int64_t n,
                        const Plan& pl, hipStream_t st)
{
    if (n <= pl.block) return closure(ctx, dt, D, ld, off, n, pl.closure, st);
    if (pl.cutover > 0 && n <= pl.cutover) return fw_window(ctx, dt, D, ld, off, n, pl, st);
    // split point: half, rounded up to a multiple of the leaf size (so every
    // leaf and every sub-view starts on a tile boundary)
    int64_t n1 = (n + 1) / 2;
    n1 = (n1 + pl.block - 1) / pl.block * pl.block;
    if (n1 >= n) n1 = n - 1;
    const int64_t n2 = n - n1;
    const int64_t a = off, d = off + n1;
    apsp_status_t rc;
    // A <- A*
    if ((rc = rk_window(ctx, dt, D, ld, a, n1, pl, st))) return rc;
    // B <- min(B, A (min,+) B);  C <- min(C, C (min,+) A)
    {
        apsp::GemmProblem pb = make_problem(dt, D, ld, a, a, a, d, a, d, n1, n2, n1);
        apsp::GemmProblem pc = make_problem(dt, D, ld, d, a, a, a, d, a, n2, n1, n1);
        if (pl.det && (rc = aliased_from_copies(dt, D, ld, a, d, n1, n2, pl, pb, true, pc, false, st))) return rc;
        if ((rc = run_two(ctx, dt, pb, pc, pl, st))) return rc;
    }
    // D <- min(D, C (min,+) B)
    if ((rc = run_one(ctx, dt, make_problem(dt, D, ld, d, a, a, d, d, d, n2, n2, n1), pl, st))) return rc;
    // D <- D*
    if ((rc = rk_window(ctx, dt, D, ld, d, n2, pl, st))) return rc;
    // B <- min(B, B (min,+) D);  C <- min(C, D (min,+) C)
    {
        apsp::GemmProblem pb = make_problem(dt, D, ld, a, d, d, d, a, d, n1, n2, n2);
        apsp::GemmProblem pc = make_problem(dt, D, ld, d, d, d, a, d, a, n2, n1, n2);
        if (pl.det && (rc = aliased_from_copies(dt, D, ld, a, d, n1, n2, pl, pb, false, pc, true, st))) return rc;
        if ((rc = run_two(ctx, dt, pb, pc, pl, st))) return rc;
    }
    // A <- min(A, B (min,+) C)
    return run_one(ctx, dt, make_problem(dt, D, ld, a, d, d, a, a, a, n1, n1, n2), pl, st);
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + bbytes && y < x + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld)
{
    if (rows <= 0 || cols <= 0) return 0;
    return (size_t)(((rows - 1) * ld + cols) * 4);
}

// Squaring runs as one launch up to this size (its passes are latency-bound
// there); larger graphs take one launch and one flag read-back per pass.
constexpr int64_t kFlowSquareMaxN = 2048;
constexpr int kSquarePassesWord = 50;   // in the synchronisation block below
// tickets, pass counters, flags and pass count of the one-launch squaring
// (scratch bytes 256 .. 511)
uint32_t* square_sync(apsp_ctx_t* ctx) { return static_cast<uint32_t*>(ctx->d_scratch) + 64; }

apsp_status_t square_common(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ld,
                            const Plan& pl, hipStream_t st)
{
    if (n <= 1) return APSP_OK;
    if (!pl.p16 && !pl.skip && n <= kFlowSquareMaxN) {
        // small graph: every pass in one launch, no read-back
        if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
        ctx->square_passes = 0;
        ctx->square_passes_device = n > 2;
        return timed(ctx, APSP_KERNEL_OTHER, 0.0, 0.0, st, [&]() -> apsp_status_t {
            HIP_TRY(apsp::launch_square_flow((apsp::DType)dt, D, (int)n, ld, square_sync(ctx), ctx->num_cus, st),
                    "squaring launch");
            return APSP_OK;
        });
    }
    uint32_t* flag = static_cast<uint32_t*>(ctx->d_scratch) + 4;
    int passes = 0;
    apsp_status_t rc;
    for (;;) {
        if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
        HIP_TRY(apsp::launch_fill_u32(flag, 0u, 1, st), "flag reset");
        const int tile = pick_tile(pl, n, n);
        const double terms = (double)n * n * n;
        rc = timed(ctx, tile == apsp::TILE_64 ? APSP_KERNEL_MINPLUS_64 : APSP_KERNEL_MINPLUS_128, terms,
                   16.0 * n * n, st, [&]() -> apsp_status_t {
                       HIP_TRY(apsp::launch_square_pass(gemm_dtype(dt, pl), tile, D, n, ld, flag, pl.skip, st),
                               "squaring pass");
                       return APSP_OK;
                   });
        if (rc) return rc;
        uint32_t h = 0;
        HIP_TRY(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st), "flag copy");
        HIP_TRY(hipStreamSynchronize(st), "flag sync");
        ++passes;
        ctx->square_passes = passes;
        ctx->square_passes_device = false;
        if (!h) break;
        if (passes > 64) return fail(APSP_E_INPUT, "squaring did not converge (negative costs?)");
    }
    return APSP_OK;
}

// APSP_FLAG_PACKED16 epilogue.  The products ran in arithmetic capped at
// kCap16 = 14847; capping commutes with min and +, so every stored value below the
// cap is an exact distance, and every stored value is the length of a real
// walk (or INF) and no larger than the input entry.  If no entry reached the
// cap the result is therefore the int32 result.  Otherwise the int32 solver
// runs again on the stored matrix: it lies between the true distances and
// the input, so its closure is the true one.
template <class Redo>
apsp_status_t finish_packed16(apsp_ctx_t* ctx, int64_t n, const void* D, int64_t ld, hipStream_t st,
                              Redo&& redo)
{
    ++ctx->p16_runs;
    auto* cnt = reinterpret_cast<unsigned long long*>(static_cast<uint32_t*>(ctx->d_scratch) + 16);
    HIP_TRY(apsp::launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), 0u, 2, st), "counter reset");
    HIP_TRY(apsp::launch_count_ge(static_cast<const uint32_t*>(D), n, ld, apsp::kCap16, cnt, st), "cap count");
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, st), "cap count copy");
    HIP_TRY(hipStreamSynchronize(st), "cap count sync");
    if (!h) return APSP_OK;
    ++ctx->p16_redone;
    return redo();
}

apsp_status_t check_packed16(apsp_dtype_t dt, const apsp_opts_t* o)
{
    if ((o->flags & APSP_FLAG_PACKED16) && dt != APSP_I32)
        return fail(APSP_E_UNSUPPORTED, "APSP_FLAG_PACKED16 needs int32 data");
    return APSP_OK;
}

apsp_status_t reject_packed16(const apsp_opts_t* o, const char* who)
{
    if (o->flags & APSP_FLAG_PACKED16)
        return fail(APSP_E_UNSUPPORTED, "APSP_FLAG_PACKED16 is not available for %s", who);
    return APSP_OK;
}

// Candidate plans scored by the cost model and timed by the autotuner.
// The last three run their products in capped 16-bit arithmetic (int32 only;
// same result, faster when every distance is below the cap, slower when the
// int32 redo runs).
struct Candidate {
    int32_t algo, block, tile, closure, cutover, flags;
};
const Candidate kCandidates[] = {
    {APSP_ALGO_FW, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 0, 0},        // size rule, n <= 4096
    {APSP_ALGO_FW, 64, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 0, 0},
    {APSP_ALGO_RKLEENE, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 0, 0},
    {APSP_ALGO_RKLEENE, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 4096, 0},  // size rule, n > 4096
    {APSP_ALGO_RKLEENE, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 1024, 0},
    {APSP_ALGO_RKLEENE, 128, APSP_TILE_64, APSP_CLOSURE_KLOOP, 0, 0},
    {APSP_ALGO_SQUARE, 0, APSP_TILE_AUTO, APSP_CLOSURE_AUTO, 0, 0},
    {APSP_ALGO_FW, 128, APSP_TILE_AUTO, APSP_CLOSURE_SQUARE, 0, 0},
    {APSP_ALGO_FW, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 0, APSP_FLAG_PACKED16},
    {APSP_ALGO_RKLEENE, 128, APSP_TILE_AUTO, APSP_CLOSURE_KLOOP, 4096, APSP_FLAG_PACKED16},
    {APSP_ALGO_SQUARE, 0, APSP_TILE_AUTO, APSP_CLOSURE_AUTO, 0, APSP_FLAG_PACKED16},
};
constexpr int32_t kNumCandidates = (int32_t)(sizeof(kCandidates) / sizeof(kCandidates[0]));

// Candidate plans of apsp_batched (scored by the cost model's last outputs):
// schedule flags, round width of the large graphs, sub-tiled products
// (tile = APSP_TILE_64), and the n above which a graph counts as large.
struct BatchCandidate {
    int32_t flags, block, tile, split;
};
const BatchCandidate kBatchCandidates[] = {
    {APSP_FLAG_BATCH_LOCKSTEP, 0, 0, 0},                    // lock-step, 128-wide rounds
    {APSP_FLAG_BATCH_QUEUE, 128, 0, 0},                     // queue, whole 128-tiles
    {APSP_FLAG_BATCH_QUEUE, 128, APSP_TILE_64, 128},        // queue, 64 x 64 sub-tiles for n > 128
    {APSP_FLAG_BATCH_QUEUE, 128, APSP_TILE_64, 256},        // queue, 64 x 64 sub-tiles for n > 256
    {APSP_FLAG_BATCH_QUEUE, 64, 0, 384},                    // queue, 64-wide rounds for n > 384
    {APSP_FLAG_BATCH_PERSISTENT, 0, 0, 0},                  // persistent, one workgroup per graph
};
constexpr int32_t kNumBatchCandidates = (int32_t)(sizeof(kBatchCandidates) / sizeof(kBatchCandidates[0]));
constexpr int32_t kDefaultBatchCandidate = 2;   // without a cost model

void batch_candidate_opts(int32_t i, apsp_opts_t* out)
{
    *out = apsp_opts_t{};
    const BatchCandidate& c = kBatchCandidates[i];
    out->flags = c.flags;
    out->block = c.block;
    out->tile = c.tile;
    out->reserved[0] = c.split;
}
constexpr int32_t kCmMaxRows = 4096;

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void free_costmodel(apsp_ctx_t* c)
{
    for (float** p : {&c->cm_params, &c->cm_m, &c->cm_v, &c->cm_grad, &c->cm_ws, &c->cm_io}) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    c->cm_K = 0;
}

apsp_status_t check_model(apsp_ctx_t* ctx)
{
    if (!ctx->cm_params) return fail(APSP_E_STATE, "no cost model: call apsp_costmodel_init first");
    return APSP_OK;
}

// Automatic choice of the predecessor form: the sparse one does n * m
// candidate updates (each an LDS atomic) against the dense kernel's n^3
// argmin terms, so it is used while the edges are a small share of n^2.
constexpr double kPredSparseMaxDensity = 0.25;
constexpr int64_t kPredSparseMaxN = 65535;


// ---------------------------------------------------------------------------
// Caller workspace (apsp_set_workspace): the only device memory a compute
// call uses beyond its arguments and the context's 4 KB scratch.
// ---------------------------------------------------------------------------
constexpr size_t kWsAlign = 256;
enum { WS_NONE = 0, WS_BATCHED = 1, WS_PRED = 2 };

size_t align_up(size_t x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

// Sparse predecessors: [use-sparse flag][edge counts][offsets + range
// starts][edge list]; the edge list takes whatever room is left.
struct PredLayout {
    size_t counts, offsets, edges;   // byte offsets; edges = size of the fixed part
};
PredLayout pred_layout(int64_t n)
{
    const int64_t nr = apsp::pred_sparse_ranges((int32_t)n);
    const size_t cells = (size_t)nr * (size_t)n;
    PredLayout L;
    L.counts = kWsAlign;
    L.offsets = L.counts + align_up(cells * sizeof(int32_t));
    L.edges = L.offsets + align_up((cells + (size_t)nr + 1) * sizeof(int64_t));
    return L;
}
size_t pred_ws_bytes(int64_t n)
{
    // room for every edge the automatic choice would still take sparse
    const double m = kPredSparseMaxDensity * (double)n * (double)n;
    return pred_layout(n).edges + align_up((size_t)m * sizeof(uint64_t));
}

// Planner feature pass of apsp_solve / apsp_features: a union-find parent
// per vertex (counters in the context scratch).
size_t solve_ws_bytes(int64_t n) { return kWsAlign + align_up((size_t)n * sizeof(int32_t)); }

// APSP_FLAG_DETERMINISTIC: R-Kleene's top-level B and C copies (2 n1 n2 <=
// 2 floor(n^2 / 4) elements for any split n1 + n2 = n) or blocked FW's panel
// copies (2 x 128 x n), whichever is larger; the recursion reuses the same
// memory in stream order.
size_t det_ws_bytes(int64_t n)
{
    if (n <= 1) return 0;
    return align_up((size_t)std::max<int64_t>(2 * ((n * n) / 4), 2 * 128 * n) * sizeof(int32_t));
}

// Points the plan at the workspace for the deterministic copies, or fails.
apsp_status_t det_workspace(apsp_ctx_t* ctx, int64_t n, Plan& pl)
{
    if (!pl.det) return APSP_OK;
    const size_t need = det_ws_bytes(n);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(APSP_E_NOMEM, "APSP_FLAG_DETERMINISTIC needs a workspace of %zu bytes (apsp_workspace_size)", need);
    pl.tmp = ctx->ws;
    ctx->ws_owner = WS_NONE;
    return APSP_OK;
}

// Batched plan: [pointer record][ticket, error word][queue order]
// [lock-step items][queue tasks][queue counters], each part 256-aligned.
struct BatchLayout {
    size_t ticket, err, qoff, order, items, tasks, counters, bytes;
};
constexpr int kMaxXcds = 8;
BatchLayout batch_layout(int32_t count, size_t items, size_t tasks, int32_t counters)
{
    BatchLayout L;
    L.ticket = kWsAlign;                                   // one 256-byte slot per XCD queue
    L.err = L.ticket + kMaxXcds * kWsAlign;
    L.qoff = L.err + kWsAlign;
    L.order = L.qoff + kWsAlign;
    L.items = L.order + align_up((size_t)count * sizeof(int32_t));
    L.tasks = L.items + align_up(items * sizeof(int4));
    L.counters = L.tasks + align_up(tasks * sizeof(apsp::BatchTask));
    L.bytes = L.counters + align_up((size_t)std::max(counters, 1) * sizeof(int32_t));
    return L;
}
// XCDs of the device: MI355X has 8 XCDs of 32 CUs (a partitioned device
// exposes fewer CUs and so fewer XCDs).
int num_xcds(const apsp_ctx_t* ctx) { return std::max(1, std::min(kMaxXcds, ctx->num_cus / 32)); }

// Per-graph plan of the queue schedule: graphs with n > opts->reserved[0]
// (every graph when it is 0) take round width opts->block (0: 128) and, with
// opts->tile = APSP_TILE_64, products cut into 64 x 64 sub-tile tasks; the
// others take 128-wide rounds of whole tiles.
int queue_width(const apsp_opts_t* o, int n)
{
    const int wide = o->block ? o->block : 128;
    return n > o->reserved[0] ? wide : 128;
}
int queue_sub(const apsp_opts_t* o, int n)
{
    return (n > o->reserved[0] && o->tile == APSP_TILE_64 && queue_width(o, n) == 128) ? 64 : 0;
}

// Upper bounds per graph of n <= max_n (nb 128-wide rounds): lock-step
// items, queue tasks, queue counters.
int64_t batched_rounds(int max_n)
{
    const int64_t B = apsp::batched_round_width();
    return (max_n + B - 1) / B;
}
size_t batched_items_bound(int max_n)
{
    const int64_t nb = batched_rounds(max_n);
    return (size_t)(1 + nb * (2 * (nb - 1) + 1 + 4 * nb * nb));
}
// queue tasks and counters: bounded by the narrowest round width (64)
int64_t queue_rounds_bound(int max_n) { return (max_n + 63) / 64; }
size_t batched_tasks_bound(int max_n)
{
    const int64_t nb = queue_rounds_bound(max_n);
    return (size_t)(1 + nb * (2 * (nb - 1) + 1 + nb * nb));
}

// Drops the captured batched launches (after the stream has drained them).
void drop_batch_graphs(apsp_ctx_t* ctx)
{
    if (ctx->bexec) hipGraphExecDestroy(ctx->bexec);
    if (ctx->bgraph) hipGraphDestroy(ctx->bgraph);
    if (ctx->lexec) hipGraphExecDestroy(ctx->lexec);
    if (ctx->lgraph) hipGraphDestroy(ctx->lgraph);
    ctx->bexec = nullptr;
    ctx->bgraph = nullptr;
    ctx->bnode = nullptr;
    ctx->lexec = nullptr;
    ctx->lgraph = nullptr;
    if (ctx->qexec) hipGraphExecDestroy(ctx->qexec);
    if (ctx->qgraph) hipGraphDestroy(ctx->qgraph);
    ctx->qexec = nullptr;
    ctx->qgraph = nullptr;
}

// Device addresses of the fixed scratch, one per GPU, and the serial of the
// last plan uploaded into each (calls on one GPU share the array).
struct FixedScratch {
    char* ptr = nullptr;
    uint64_t serial = 0;
};
std::mutex g_fixed_mu;
std::map<int, FixedScratch> g_fixed;
uint64_t g_fixed_next = 0;

// Called with `device` current.
apsp_status_t fixed_scratch_address(int device, char** out)
{
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    FixedScratch& f = g_fixed[device];
    if (!f.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "fixed scratch address");
        f.ptr = static_cast<char*>(p);
    }
    *out = f.ptr;
    return APSP_OK;
}

bool fixed_plan_resident(apsp_ctx_t* ctx)
{
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    return ctx->fixed_serial != 0 && g_fixed[ctx->device].serial == ctx->fixed_serial;
}

void fixed_plan_claim(apsp_ctx_t* ctx)
{
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    ctx->fixed_serial = ++g_fixed_next;
    g_fixed[ctx->device].serial = ctx->fixed_serial;
}


// Scratch words of the feature pass (bytes 192..207 of the context scratch).
unsigned long long* feat_edges(apsp_ctx_t* ctx)
{
    return reinterpret_cast<unsigned long long*>(static_cast<char*>(ctx->d_scratch) + 192);
}
uint32_t* feat_roots(apsp_ctx_t* ctx) { return reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->d_scratch) + 200); }

// A model scores the single-graph candidates when it has at least their K
// outputs, and the batch candidates when it has both sets (batch outputs last).
bool model_ready(const apsp_ctx_t* ctx) { return ctx->cm_params && ctx->cm_K >= kNumCandidates; }
bool batch_model_ready(const apsp_ctx_t* ctx)
{
    return ctx->cm_params && ctx->cm_K == kNumCandidates + kNumBatchCandidates;
}

// First minimum of the predicted scores among the candidates `dt` can run.
int32_t pick_candidate(apsp_dtype_t dt, const float* pred)
{
    int32_t choice = -1;
    for (int32_t i = 0; i < kNumCandidates; ++i) {
        if (dt != APSP_I32 && (kCandidates[i].flags & APSP_FLAG_PACKED16)) continue;
        if (choice < 0 || pred[i] < pred[choice]) choice = i;
    }
    return choice;
}

// Cost-model plan for one matrix, on the device: the feature pass writes
// the four inputs next to the model's outputs, the forward pass scores every
// candidate, and one read-back (the stream is synchronised) returns both.
apsp_status_t plan_matrix(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, const void* D, int64_t ld, hipStream_t st,
                          float* h_x, int32_t* h_choice)
{
    float* x = ctx->cm_io;
    const int K = ctx->cm_K;
    HIP_TRY(apsp::launch_graph_features((apsp::DType)dt, D, (int32_t)n, ld, reinterpret_cast<int32_t*>(ctx->ws),
                                        feat_edges(ctx), feat_roots(ctx), x, st),
            "feature pass");
    HIP_TRY(apsp::launch_mlp_forward(ctx->cm_params, ctx->cm_norm, x, 1, K, ctx->cm_ws, x + 4, st), "mlp forward");
    float* h = ctx->h_io;   // pinned; 4 + K <= 1024 floats
    HIP_TRY(hipMemcpyAsync(h, x, (4 + K) * sizeof(float), hipMemcpyDeviceToHost, st), "plan read-back");
    HIP_TRY(hipStreamSynchronize(st), "plan sync");
    if (h_x) std::copy(h, h + 4, h_x);
    *h_choice = pick_candidate(dt, h + 4);
    return APSP_OK;
}

bool opts_all_auto(const apsp_opts_t* o)
{
    return o->algo == APSP_ALGO_AUTO && !o->block && !o->tile && !o->closure && !o->cutover && !o->flags;
}
}  // namespace

extern "C" {

const char* apsp_last_error(void) { return g_last_error.c_str(); }

const char* apsp_version(void) { return "apsp-mi355x 0.1 (gfx950)"; }

apsp_status_t apsp_create(apsp_ctx_t** out, int32_t device)
{
    if (!out) return fail(APSP_E_ARG, "ctx output pointer is NULL");
    *out = nullptr;
    if (device < 0) return fail(APSP_E_ARG, "device = %d", device);
    if (fault_injected("create")) return fail(APSP_E_HIP, "injected create failure");
    if (fault_injected("hostctx")) {
        // host-side tests without a GPU: a context with no device resources,
        // enough for the checks a call makes before its first HIP call
        apsp_ctx_t* c = new apsp_ctx_t();
        c->device = device;
        *out = c;
        return APSP_OK;
    }
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (device >= count) return fail(APSP_E_ARG, "device %d of %d", device, count);
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    char* fixed = nullptr;
    apsp_status_t frc = fixed_scratch_address(device, &fixed);
    if (frc) return frc;
    apsp_ctx_t* c = new apsp_ctx_t();
    c->device = device;
    c->fixed = fixed;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(APSP_E_HIP, "capture stream creation failed");
    }
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_p, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming) != hipSuccess) {
        if (c->side) hipStreamDestroy(c->side);
        if (c->ev_a) hipEventDestroy(c->ev_a);
        if (c->ev_p) hipEventDestroy(c->ev_p);
        if (c->ev_b) hipEventDestroy(c->ev_b);
        hipStreamDestroy(c->capture);
        delete c;
        return fail(APSP_E_HIP, "look-ahead stream creation failed");
    }
    c->scratch_bytes = 4096;
    hipError_t e = hipMalloc(&c->d_scratch, c->scratch_bytes);
    if (e != hipSuccess) {
        hipStreamDestroy(c->capture);
        hipStreamDestroy(c->side);
        hipEventDestroy(c->ev_a);
        hipEventDestroy(c->ev_p);
        hipEventDestroy(c->ev_b);
        delete c;
        return fail(APSP_E_NOMEM, "scratch allocation: %s", hipGetErrorString(e));
    }
    // pinned, so that the plan read-back is one direct copy
    e = hipHostMalloc(reinterpret_cast<void**>(&c->h_io), 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(c->d_scratch);
        hipStreamDestroy(c->capture);
        hipStreamDestroy(c->side);
        hipEventDestroy(c->ev_a);
        hipEventDestroy(c->ev_p);
        hipEventDestroy(c->ev_b);
        delete c;
        return fail(APSP_E_NOMEM, "pinned host buffer: %s", hipGetErrorString(e));
    }
    *out = c;
    return APSP_OK;
}

apsp_status_t apsp_destroy(apsp_ctx_t* ctx)
{
    if (!ctx) return APSP_OK;
    if (ctx->magic != 0x41505350) return fail(APSP_E_STATE, "context is not valid");
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    if (ctx->d_scratch) hipFree(ctx->d_scratch);
    if (ctx->h_io) hipHostFree(ctx->h_io);
    for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
    free_costmodel(ctx);
    drop_batch_graphs(ctx);
    if (ctx->capture) hipStreamDestroy(ctx->capture);
    if (ctx->side) hipStreamDestroy(ctx->side);
    if (ctx->ev_a) hipEventDestroy(ctx->ev_a);
    if (ctx->ev_p) hipEventDestroy(ctx->ev_p);
    if (ctx->ev_b) hipEventDestroy(ctx->ev_b);
    ctx->magic = 0;
    delete ctx;
    return APSP_OK;
}

size_t apsp_workspace_size(apsp_ctx_t* ctx, int32_t op, apsp_dtype_t dt, int64_t n_or_total, int32_t count)
{
    if (check_ctx(ctx) || check_dtype(dt)) return 0;
    if (n_or_total < 0 || count < 0) {
        fail(APSP_E_ARG, "negative size");
        return 0;
    }
    switch (op) {
    case APSP_OP_SOLVE: return n_or_total > 1 ? solve_ws_bytes(n_or_total) : 0;
    case APSP_OP_BATCHED: {
        // lock-step items up to the lock-step limit, queue tasks and counters
        // up to the queue limit
        const int items_n = (int)std::max<int64_t>(std::min<int64_t>(n_or_total, apsp::batched_max_n()), 1);
        const int queue_n = (int)std::max<int64_t>(std::min<int64_t>(n_or_total, apsp::kQueueMaxN), 1);
        const int32_t nb = (int32_t)queue_rounds_bound(queue_n);
        return batch_layout(count, (size_t)count * batched_items_bound(items_n),
                            (size_t)count * batched_tasks_bound(queue_n),
                            count * (nb >= 2 ? 4 * nb : 0) + kMaxXcds * (int32_t)(kWsAlign / sizeof(int32_t)))
            .bytes;
    }
    case APSP_OP_PREDECESSORS:
        if (n_or_total <= 1 || n_or_total > kPredSparseMaxN) return 0;
        return pred_ws_bytes(n_or_total);
    case APSP_OP_DETERMINISTIC: return det_ws_bytes(n_or_total);
    default:
        fail(APSP_E_ARG, "op = %d", op);
        return 0;
    }
}

apsp_status_t apsp_set_workspace(apsp_ctx_t* ctx, void* d_ptr, size_t bytes)
{
    apsp_status_t rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (bytes > 0 && !d_ptr) return fail(APSP_E_ARG, "workspace pointer is NULL");
    if (d_ptr && (reinterpret_cast<uintptr_t>(d_ptr) % kWsAlign) != 0)
        return fail(APSP_E_ARG, "workspace must be %zu-byte aligned", kWsAlign);
    if (d_ptr == ctx->ws && bytes == ctx->ws_bytes) return APSP_OK;
    // captured batched launches point into the old workspace: let any that
    // are still running finish before they are destroyed
    if (ctx->bexec || ctx->lexec || ctx->qexec) HIP_TRY(hipDeviceSynchronize(), "workspace change sync");
    drop_batch_graphs(ctx);
    ctx->bkey = 0;
    ctx->bcount = 0;
    ctx->bauto_key = 0;
    ctx->batch_err = nullptr;
    ctx->ws = bytes ? static_cast<char*>(d_ptr) : nullptr;
    ctx->ws_bytes = bytes;
    ctx->ws_owner = WS_NONE;
    return APSP_OK;
}

apsp_status_t minplus_gemm(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t m, int64_t n, int64_t k,
                           const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                           const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = reject_packed16(o, "minplus_gemm"))) return rc;
    if (m < 0 || n < 0 || k < 0) return fail(APSP_E_ARG, "negative size m=%lld n=%lld k=%lld",
                                             (long long)m, (long long)n, (long long)k);
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > INT32_MAX / 2) return fail(APSP_E_ARG, "size too large");
    if (m == 0 || n == 0 || k == 0) return check_ctx(ctx);
    if (!A || !B || !C) return fail(APSP_E_ARG, "NULL matrix pointer");
    if (lda < k) return fail(APSP_E_ARG, "lda = %lld < k = %lld", (long long)lda, (long long)k);
    if (ldb < n) return fail(APSP_E_ARG, "ldb = %lld < n = %lld", (long long)ldb, (long long)n);
    if (ldc < n) return fail(APSP_E_ARG, "ldc = %lld < n = %lld", (long long)ldc, (long long)n);
    const size_t cb = span_bytes(m, n, ldc);
    if (overlaps(C, cb, A, span_bytes(m, k, lda)) || overlaps(C, cb, B, span_bytes(k, n, ldb)))
        return fail(APSP_E_ARG, "C overlaps A or B");
    if ((rc = check_ctx(ctx))) return rc;
    const Plan pl = resolve(o);
    apsp::GemmProblem p{};
    p.A = A; p.B = B; p.C = C;
    p.lda = lda; p.ldb = ldb; p.ldc = ldc;
    p.M = (int32_t)m; p.N = (int32_t)n; p.K = (int32_t)k;
    return run_one(ctx, dt, p, pl, static_cast<hipStream_t>(stream));
}

apsp_status_t apsp_closure(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ldd,
                           const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = reject_packed16(o, "apsp_closure")) || (rc = check_ctx(ctx))) return rc;
    if (n > 128) return fail(APSP_E_UNSUPPORTED, "closure block n = %lld > 128", (long long)n);
    if (n <= 1) return APSP_OK;
    const Plan pl = resolve(o);
    return closure(ctx, dt, D, ldd, 0, n, pl.closure, static_cast<hipStream_t>(stream));
}

apsp_status_t apsp_fw(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ldd,
                      const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = check_packed16(dt, o)) || (rc = check_ctx(ctx))) return rc;
    if (n <= 1) return APSP_OK;
    Plan pl = resolve(o);
    if ((rc = det_workspace(ctx, n, pl))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = fw_window(ctx, dt, D, ldd, 0, n, pl, st)) || !pl.p16) return rc;
    return finish_packed16(ctx, n, D, ldd, st, [&] {
        pl.p16 = false;
        return fw_window(ctx, dt, D, ldd, 0, n, pl, st);
    });
}

apsp_status_t apsp_rkleene(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ldd,
                           const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = check_packed16(dt, o)) || (rc = check_ctx(ctx))) return rc;
    if (n <= 1) return APSP_OK;
    Plan pl = resolve(o);
    if ((rc = det_workspace(ctx, n, pl))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = rk_window(ctx, dt, D, ldd, 0, n, pl, st)) || !pl.p16) return rc;
    return finish_packed16(ctx, n, D, ldd, st, [&] {
        pl.p16 = false;
        return rk_window(ctx, dt, D, ldd, 0, n, pl, st);
    });
}

apsp_status_t apsp_square(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ldd,
                          const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = check_packed16(dt, o)) || (rc = check_ctx(ctx))) return rc;
    if (o->flags & APSP_FLAG_DETERMINISTIC)
        return fail(APSP_E_UNSUPPORTED, "apsp_square has no deterministic mode (use apsp_fw or apsp_rkleene)");
    if (n <= 1) return APSP_OK;
    Plan pl = resolve(o);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = square_common(ctx, dt, n, D, ldd, pl, st)) || !pl.p16) return rc;
    return finish_packed16(ctx, n, D, ldd, st, [&] {
        pl.p16 = false;
        return square_common(ctx, dt, n, D, ldd, pl, st);
    });
}

apsp_status_t apsp_square_passes(apsp_ctx_t* ctx, void* stream, int32_t* h_passes)
{
    apsp_status_t rc;
    if (!h_passes) return fail(APSP_E_ARG, "h_passes is NULL");
    if ((rc = check_ctx(ctx))) return rc;
    if (ctx->square_passes < 0) return fail(APSP_E_STATE, "apsp_square has not run on this context");
    if (!ctx->square_passes_device) {
        *h_passes = ctx->square_passes;
        return APSP_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ctx->h_io, square_sync(ctx) + kSquarePassesWord, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           st),
            "pass count read-back");
    HIP_TRY(hipStreamSynchronize(st), "pass count sync");
    *h_passes = (int32_t)reinterpret_cast<const uint32_t*>(ctx->h_io)[0];
    return APSP_OK;
}

apsp_status_t apsp_packed16_counts(apsp_ctx_t* ctx, int64_t* runs, int64_t* redone)
{
    apsp_status_t rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!runs || !redone) return fail(APSP_E_ARG, "NULL output pointer");
    *runs = ctx->p16_runs;
    *redone = ctx->p16_redone;
    return APSP_OK;
}

apsp_status_t apsp_solve(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, void* D, int64_t ldd,
                         const apsp_opts_t* opts, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = check_packed16(dt, o)) || (rc = check_ctx(ctx))) return rc;
    switch (o->algo) {
    case APSP_ALGO_FW: return apsp_fw(ctx, dt, n, D, ldd, o, stream);
    case APSP_ALGO_SQUARE: return apsp_square(ctx, dt, n, D, ldd, o, stream);
    case APSP_ALGO_RKLEENE: return apsp_rkleene(ctx, dt, n, D, ldd, o, stream);
    default: {
        // all options automatic, a cost model for the candidate table loaded
        // and a workspace for the feature pass: the model's pick
        if (opts_all_auto(o) && n > 1 && model_ready(ctx) && ctx->ws && ctx->ws_bytes >= solve_ws_bytes(n)) {
            int32_t choice = -1;
            if ((rc = plan_matrix(ctx, dt, n, D, ldd, static_cast<hipStream_t>(stream), nullptr, &choice))) return rc;
            ctx->ws_owner = WS_NONE;
            apsp_opts_t po;
            if ((rc = apsp_candidate(choice, &po))) return rc;
            ctx->last_choice = choice;
            return apsp_solve(ctx, dt, n, D, ldd, &po, stream);
        }
        ctx->last_choice = -1;
        // size rule: R-Kleene's top-level products are large and efficient;
        // blocked FW has fewer launches and wins up to about n = 4096, so it
        // also closes R-Kleene's sub-problems of that size
        if (n <= 4096) return apsp_fw(ctx, dt, n, D, ldd, o, stream);
        apsp_opts_t o2 = *o;
        if (!o2.cutover) o2.cutover = 4096;
        return apsp_rkleene(ctx, dt, n, D, ldd, &o2, stream);
    }
    }
}

apsp_status_t apsp_predecessors_ex(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, const void* D, int64_t ldd,
                                   const void* W, int64_t ldw, int32_t* P, int64_t ldp, int32_t method,
                                   void* stream)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd)) || (rc = check_square(n, W, ldw)) ||
        (rc = check_square(n, P, ldp)))
        return rc;
    if (n > INT32_MAX / 2) return fail(APSP_E_ARG, "n too large");
    if (method < APSP_PRED_AUTO || method > APSP_PRED_SPARSE) return fail(APSP_E_ARG, "method = %d", method);
    const size_t pb = span_bytes(n, n, ldp);
    if (n > 0 && (overlaps(P, pb, D, span_bytes(n, n, ldd)) || overlaps(P, pb, W, span_bytes(n, n, ldw))))
        return fail(APSP_E_ARG, "P overlaps D or W");
    if (method == APSP_PRED_SPARSE && n > kPredSparseMaxN)
        return fail(APSP_E_UNSUPPORTED, "sparse predecessors need n <= %lld", (long long)kPredSparseMaxN);
    if ((rc = check_ctx(ctx))) return rc;
    if (n == 0) return APSP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the sparse form needs the workspace's fixed part (flag, counts, offsets)
    const PredLayout L = pred_layout(n);
    const bool sparse_possible = method != APSP_PRED_DENSE && n <= kPredSparseMaxN;
    const bool have_ws = ctx->ws && ctx->ws_bytes > L.edges;
    if (method == APSP_PRED_SPARSE && !have_ws)
        return fail(APSP_E_NOMEM, "sparse predecessors need a workspace of more than %zu bytes (apsp_workspace_size)",
                    L.edges);
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    auto dense = [&](const uint32_t* skip_if_set) -> apsp_status_t {
        const double terms = (double)n * n * n;
        return timed(ctx, APSP_KERNEL_OTHER, terms, 12.0 * n * n, st, [&]() -> apsp_status_t {
            HIP_TRY(apsp::launch_predecessors((apsp::DType)dt, D, ldd, W, ldw, P, ldp, (int32_t)n, skip_if_set, st),
                    "predecessor launch");
            return APSP_OK;
        });
    };
    if (!sparse_possible || !have_ws) return dense(nullptr);
    // On the device: count each row's edges per column range, scan the counts
    // into the edge-list layout and decide -- sparse when the list fits the
    // workspace (and, for the automatic choice, m <= n^2/4), else dense.
    // Both forms are enqueued; the one not chosen returns at once, so nothing
    // is read back and the call only enqueues.
    uint32_t* flag = reinterpret_cast<uint32_t*>(ctx->ws);
    int32_t* counts = reinterpret_cast<int32_t*>(ctx->ws + L.counts);
    int64_t* offs = reinterpret_cast<int64_t*>(ctx->ws + L.offsets);
    uint64_t* edges = reinterpret_cast<uint64_t*>(ctx->ws + L.edges);
    const int64_t cells = (int64_t)apsp::pred_sparse_ranges((int32_t)n) * n;
    const int64_t edge_cap = (int64_t)((ctx->ws_bytes - L.edges) / sizeof(uint64_t));
    const int64_t dense_limit = method == APSP_PRED_AUTO ? (int64_t)(kPredSparseMaxDensity * (double)n * (double)n)
                                                         : INT64_MAX;
    ctx->ws_owner = WS_PRED;
    apsp_status_t rc2 = timed(ctx, APSP_KERNEL_OTHER, 0.0, 8.0 * n * n, st, [&]() -> apsp_status_t {
        HIP_TRY(apsp::launch_edge_count((apsp::DType)dt, W, ldw, (int32_t)n, counts, st), "edge count launch");
        HIP_TRY(apsp::launch_edge_scan(counts, (int32_t)n, offs, edge_cap, dense_limit, flag, st), "edge scan launch");
        HIP_TRY(apsp::launch_pred_sparse((apsp::DType)dt, D, ldd, W, ldw, P, ldp, (int32_t)n, offs, offs + cells, edges,
                                         flag, st),
                "sparse predecessor launch");
        return APSP_OK;
    });
    if (rc2) return rc2;
    return dense(flag);
}

apsp_status_t apsp_predecessors(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, const void* D, int64_t ldd,
                                const void* W, int64_t ldw, int32_t* P, int64_t ldp, void* stream)
{
    return apsp_predecessors_ex(ctx, dt, n, D, ldd, W, ldw, P, ldp, APSP_PRED_AUTO, stream);
}


apsp_status_t apsp_path(apsp_ctx_t* ctx, int64_t n, const int32_t* P, int64_t ldp, int32_t count,
                        const int32_t* d_src, const int32_t* d_dst, int32_t* d_paths, int32_t max_len,
                        int32_t* d_len, void* stream)
{
    apsp_status_t rc;
    if ((rc = check_square(n, P, ldp))) return rc;
    if (n > INT32_MAX) return fail(APSP_E_ARG, "n too large");
    if (count < 0) return fail(APSP_E_ARG, "count = %d is negative", count);
    if (max_len < 1) return fail(APSP_E_ARG, "max_len = %d (>= 1)", max_len);
    if (count > 0 && (!d_src || !d_dst || !d_paths || !d_len)) return fail(APSP_E_ARG, "NULL query pointer");
    if ((rc = check_ctx(ctx))) return rc;
    if (count == 0) return APSP_OK;
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    HIP_TRY(apsp::launch_paths(P, ldp, (int32_t)n, count, d_src, d_dst, d_paths, max_len, d_len,
                               static_cast<hipStream_t>(stream)),
            "path launch");
    return APSP_OK;
}

apsp_status_t apsp_features(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, const void* D, int64_t ldd, void* stream,
                            float* h_features)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    if (!h_features) return fail(APSP_E_ARG, "h_features is NULL");
    if (n > INT32_MAX) return fail(APSP_E_ARG, "n too large");
    if ((rc = check_ctx(ctx))) return rc;
    const size_t need = n > 1 ? solve_ws_bytes(n) : 0;
    if (need && (!ctx->ws || ctx->ws_bytes < need))
        return fail(APSP_E_NOMEM, "apsp_features needs a workspace of %zu bytes (apsp_workspace_size)", need);
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* x = reinterpret_cast<float*>(static_cast<char*>(ctx->d_scratch) + 208);
    int32_t* parent = n > 1 ? reinterpret_cast<int32_t*>(ctx->ws) : nullptr;
    if (n > 1) ctx->ws_owner = WS_NONE;
    HIP_TRY(apsp::launch_graph_features((apsp::DType)dt, D, (int32_t)std::max<int64_t>(n, 0), ldd, parent,
                                        feat_edges(ctx), feat_roots(ctx), x, st),
            "feature pass");
    HIP_TRY(hipMemcpyAsync(h_features, x, 4 * sizeof(float), hipMemcpyDeviceToHost, st), "feature read-back");
    HIP_TRY(hipStreamSynchronize(st), "feature sync");
    return APSP_OK;
}

apsp_status_t apsp_solve_choice(apsp_ctx_t* ctx, int32_t* h_choice)
{
    apsp_status_t rc;
    if (!h_choice) return fail(APSP_E_ARG, "h_choice is NULL");
    if ((rc = check_ctx(ctx))) return rc;
    *h_choice = ctx->last_choice;
    return APSP_OK;
}

apsp_status_t apsp_validate(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, const void* D, int64_t ldd,
                            void* stream, int64_t* h_violations)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt)) || (rc = check_square(n, D, ldd))) return rc;
    if (!h_violations) return fail(APSP_E_ARG, "h_violations is NULL");
    if ((rc = check_ctx(ctx))) return rc;
    *h_violations = 0;
    if (n == 0) return APSP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    unsigned long long* cnt = static_cast<unsigned long long*>(ctx->d_scratch);
    HIP_TRY(apsp::launch_validate((apsp::DType)dt, D, n, ldd, cnt, st), "validate launch");
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, st), "validate copy");
    HIP_TRY(hipStreamSynchronize(st), "validate sync");
    *h_violations = (int64_t)h;
    if (h) return fail(APSP_E_INPUT, "%llu entries violate the input contract", h);
    return APSP_OK;
}

}  // extern "C"

namespace {

// The cost model's four inputs for a batch: log2 of the largest n, log10 of
// the batch's density (edges / sum of n (n - 1), clamped to 1e-9), log2 of
// the graph count, and the share of the batch's work (sum of n^3) in graphs
// with n > 256.
void batch_features(int32_t count, const int32_t* h_sizes, double density, float* x)
{
    int32_t nmax = 1;
    double all = 0.0, big = 0.0;
    for (int32_t g = 0; g < count; ++g) {
        nmax = std::max(nmax, h_sizes[g]);
        const double w = (double)h_sizes[g] * h_sizes[g] * h_sizes[g];
        all += w;
        if (h_sizes[g] > 256) big += w;
    }
    x[0] = (float)std::log2((double)nmax);
    x[1] = (float)std::log10(std::max(density, 1e-9));
    x[2] = (float)std::log2((double)std::max(count, 1));
    x[3] = (float)(all > 0.0 ? big / all : 0.0);
}

// First minimum of the batch candidates' predicted scores (outputs
// kNumCandidates ..).
bool batch_candidate_is_queue(int32_t i) { return (kBatchCandidates[i].flags & APSP_FLAG_BATCH_QUEUE) != 0; }

// The best-scored batch candidate; queue candidates only when a graph is
// above the lock-step and persistent limit.
int32_t pick_batch_candidate(const float* pred, bool queue_only)
{
    int32_t choice = -1;
    for (int32_t i = 0; i < kNumBatchCandidates; ++i)
        if ((!queue_only || batch_candidate_is_queue(i)) && (choice < 0 || pred[i] < pred[choice])) choice = i;
    return choice;
}

// Scores the batch candidates for features x (device forward pass, one
// read-back).
apsp_status_t score_batch(apsp_ctx_t* ctx, const float* x, bool queue_only, hipStream_t st, int32_t* choice)
{
    const int K = ctx->cm_K;
    HIP_TRY(hipMemcpyAsync(ctx->cm_io, x, 4 * sizeof(float), hipMemcpyHostToDevice, st), "plan features upload");
    HIP_TRY(apsp::launch_mlp_forward(ctx->cm_params, ctx->cm_norm, ctx->cm_io, 1, K, ctx->cm_ws, ctx->cm_io + 4, st),
            "mlp forward");
    std::vector<float> h(K);
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->cm_io + 4, K * sizeof(float), hipMemcpyDeviceToHost, st), "scores read-back");
    HIP_TRY(hipStreamSynchronize(st), "plan sync");
    *choice = pick_batch_candidate(h.data() + kNumCandidates, queue_only);
    return APSP_OK;
}

// Automatic plan of apsp_batched: the cost model's pick from the batch's
// features (the density is counted on the device and read back), made once
// per batch shape; the default candidate without a model with batch outputs.
apsp_status_t batch_auto_plan(apsp_ctx_t* ctx, apsp_dtype_t dt, int32_t count, const void* data,
                              const int64_t* d_offsets, const int32_t* d_sizes, const int32_t* h_sizes,
                              hipStream_t st, apsp_opts_t* out)
{
    int32_t max_n = 0;
    for (int32_t g = 0; g < count; ++g) max_n = std::max(max_n, h_sizes[g]);
    uint64_t key = 0xcbf29ce484222325ull ^ (uint64_t)dt;
    for (int32_t g = 0; g < count; ++g) key = (key ^ (uint64_t)(uint32_t)h_sizes[g]) * 1099511628211ull;
    key = (key ^ (uint64_t)count) * 1099511628211ull;
    key ^= batch_model_ready(ctx) ? 0x9e3779b97f4a7c15ull : 0;
    if (key != ctx->bauto_key || ctx->bauto_choice < 0) {
        int32_t choice = kDefaultBatchCandidate;   // a queue candidate
        if (batch_model_ready(ctx)) {
            auto* tot = reinterpret_cast<unsigned long long*>(static_cast<char*>(ctx->d_scratch) + 224);
            HIP_TRY(apsp::launch_batch_edges((apsp::DType)dt, data, d_offsets, d_sizes, count, tot, st),
                    "batch edge count");
            unsigned long long m = 0;
            HIP_TRY(hipMemcpyAsync(&m, tot, sizeof m, hipMemcpyDeviceToHost, st), "edge count read-back");
            HIP_TRY(hipStreamSynchronize(st), "edge count sync");
            double pairs = 0.0;
            for (int32_t g = 0; g < count; ++g) pairs += (double)h_sizes[g] * std::max(h_sizes[g] - 1, 0);
            float x[4];
            batch_features(count, h_sizes, pairs > 0.0 ? (double)m / pairs : 0.0, x);
            apsp_status_t rc = score_batch(ctx, x, max_n > apsp::batched_max_n(), st, &choice);
            if (rc) return rc;
        }
        ctx->bauto_key = key;
        ctx->bauto_choice = choice;
    }
    batch_candidate_opts(ctx->bauto_choice, out);
    // fewer graphs than XCDs: one queue for the device, so every XCD works
    if ((out->flags & APSP_FLAG_BATCH_QUEUE) && count < num_xcds(ctx)) out->flags |= APSP_FLAG_BATCH_GLOBAL;
    return APSP_OK;
}

// Where a batched plan lives: the caller's workspace (apsp_batched) or the
// library's fixed device scratch (apsp_batched_noalloc, no graph replay).
struct PlanMem {
    bool fixed;   // the fixed scratch (direct launches only)
};

apsp_status_t batched_common(apsp_ctx_t* ctx, apsp_dtype_t dt, int32_t count, void* data,
                             const int64_t* d_offsets, const int32_t* d_sizes, const int32_t* h_sizes,
                             const apsp_opts_t* opts, void* stream, PlanMem pm, const char* who)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt))) return rc;
    const apsp_opts_t* o = opts_or_default(opts);
    if ((rc = check_opts(o)) || (rc = reject_packed16(o, who))) return rc;
    if (count < 0) return fail(APSP_E_ARG, "count = %d is negative", count);
    if (count > 0 && (!data || !d_offsets || !d_sizes || !h_sizes))
        return fail(APSP_E_ARG, "NULL batch pointer");
    int32_t max_n = 0;
    for (int32_t g = 0; g < count; ++g) {
        if (h_sizes[g] < 0) return fail(APSP_E_ARG, "graph %d has n = %d", g, h_sizes[g]);
        max_n = std::max(max_n, h_sizes[g]);
    }
    // the lock-step and persistent schedules take n <= batched_max_n, the
    // queue schedule n <= kQueueMaxN (the automatic plan then picks a queue)
    const bool queue_asked = (o->flags & APSP_FLAG_BATCH_QUEUE) &&
                             !(o->flags & (APSP_FLAG_BATCH_PERSISTENT | APSP_FLAG_BATCH_PER_GRAPH));
    const int32_t limit = (queue_asked || opts_all_auto(o)) ? apsp::kQueueMaxN : apsp::batched_max_n();
    if (max_n > limit)
        return fail(APSP_E_UNSUPPORTED, "a graph has n = %d > %d for this schedule (use apsp_solve)", max_n, limit);
    if ((rc = check_ctx(ctx))) return rc;
    if (count == 0) return APSP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");

    // every option automatic: the cost model's batch plan (made once per
    // batch shape), else the default candidate
    apsp_opts_t auto_opts;
    if (opts_all_auto(o)) {
        if ((rc = batch_auto_plan(ctx, dt, count, data, d_offsets, d_sizes, h_sizes, st, &auto_opts))) return rc;
        o = &auto_opts;
    }
    // plan: largest graphs first (longest-processing-time order)
    uint64_t key = 1469598103934665603ull ^ (uint64_t)dt;
    for (int32_t g = 0; g < count; ++g) key = (key ^ (uint64_t)(uint32_t)h_sizes[g]) * 1099511628211ull;
    key ^= (uint64_t)count << 40;
    key = (key ^ (uint64_t)(uint32_t)o->block) * 1099511628211ull;
    key = (key ^ (uint64_t)(uint32_t)o->reserved[0]) * 1099511628211ull;
    key = (key ^ (uint64_t)(uint32_t)o->tile) * 1099511628211ull;
    constexpr int32_t kScheduleFlags = APSP_FLAG_BATCH_QUEUE | APSP_FLAG_BATCH_LOCKSTEP | APSP_FLAG_BATCH_PERSISTENT |
                                       APSP_FLAG_BATCH_PER_GRAPH | APSP_FLAG_BATCH_GLOBAL;
    key = (key ^ (uint64_t)(uint32_t)(o->flags & kScheduleFlags)) * 1099511628211ull;
    const bool use_queue = (o->flags & APSP_FLAG_BATCH_QUEUE) &&
                           !(o->flags & (APSP_FLAG_BATCH_PERSISTENT | APSP_FLAG_BATCH_PER_GRAPH));
    const bool use_lockstep = !use_queue && !(o->flags & (APSP_FLAG_BATCH_PERSISTENT | APSP_FLAG_BATCH_PER_GRAPH));
    const bool rebuild = key != ctx->bkey || count != ctx->bcount || dt != ctx->bdtype;
    std::vector<int32_t> order;
    std::vector<int4> items;
    std::vector<apsp_ctx::Launch> launches;
    std::vector<apsp::BatchTask> qtasks;
    std::vector<int32_t> qoff;
    int32_t qcounters = 0;
    if (rebuild) {
        order.resize(count);
        for (int32_t g = 0; g < count; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return h_sizes[a] > h_sizes[b]; });
        // lock-step work items, graphs in largest-first order within each launch
        const int B = apsp::batched_round_width();
        int max_rounds = 0;
        for (int32_t g = 0; g < count; ++g) max_rounds = std::max(max_rounds, (h_sizes[g] + B - 1) / B);
        // Per round r: the pivot closures (round 0 only), the panel tiles,
        // then the remainder.  When round r+1 exists, its pivot tiles (r+1,
        // r+1) are updated and closed by one launch (phase 3) on the second
        // stream while the main stream updates every other remainder tile of
        // round r on 64 x 64 sub-tiles (phase 4); the next panels wait for
        // both.  The two streams touch disjoint tiles.
        auto add = [&](int phase, bool side, auto&& fill) {
            const int start = (int)items.size();
            for (int32_t q = 0; q < count; ++q) {
                const int32_t g = order[q];
                fill(g, (h_sizes[g] + B - 1) / B);
            }
            const int cnt = (int)items.size() - start;
            if (cnt > 0) launches.push_back({phase, start, cnt, side});
        };
        for (int r = 0; r < (use_lockstep ? max_rounds : 0); ++r) {
            if (r == 0)
                add(0, false, [&](int32_t g, int) { items.push_back(make_int4(g, 0, 0, 0)); });
            add(1, false, [&](int32_t g, int nb) {
                if (nb <= r || nb < 2) return;
                for (int t = 0; t < nb; ++t)
                    if (t != r) {
                        items.push_back(make_int4(g, r, t, 0));
                        items.push_back(make_int4(g, r, t, 1));
                    }
            });
            add(3, true, [&](int32_t g, int nb) {
                if (r + 1 < nb) items.push_back(make_int4(g, r, r + 1, r + 1));
            });
            add(4, false, [&](int32_t g, int nb) {
                if (nb <= r || nb < 2) return;
                const int n = h_sizes[g];
                for (int ti = 0; ti < nb; ++ti)
                    for (int tj = 0; tj < nb; ++tj) {
                        if (ti == r || tj == r || (ti == r + 1 && tj == r + 1)) continue;
                        // 64 x 64 sub-tiles that hold at least one entry
                        for (int si = 0; si < 2 && ti * B + si * (B / 2) < n; ++si)
                            for (int sj = 0; sj < 2 && tj * B + sj * (B / 2) < n; ++sj)
                                items.push_back(make_int4(g, r | (si << 8) | (sj << 9), ti, tj));
                    }
            });
        }
        if (use_queue) {
            std::vector<int32_t> widths(count), subs(count);
            for (int32_t g = 0; g < count; ++g) {
                widths[g] = queue_width(o, h_sizes[g]);
                subs[g] = queue_sub(o, h_sizes[g]);
            }
            // one queue per XCD, or one for the device
            const int nx = (o->flags & APSP_FLAG_BATCH_GLOBAL) ? 1 : num_xcds(ctx);
            apsp::build_xcd_queues(widths.data(), subs.data(), count, h_sizes, order, nx,
                                   (ctx->num_cus / nx) * apsp::batch_queue_resident_per_cu((apsp::DType)dt),
                                   kWsAlign / (int)sizeof(int32_t), apsp::TaskCost{}, qtasks, qoff, qcounters);
        }
    }
    // plan memory: [pointer record][ticket, error word][order][items][tasks]
    // [counters], in the caller's workspace or in the fixed scratch (after
    // its counter word)
    const BatchLayout lay = batch_layout(count, rebuild ? items.size() : ctx->litems.size(),
                                         rebuild ? qtasks.size() : ctx->qtasks.size(),
                                         rebuild ? qcounters : ctx->qcounters);
    const size_t need = lay.bytes;
    char* base;
    if (pm.fixed) {
        if (!ctx->fixed || need > kFixedScratchBytes - kWsAlign)
            return fail(APSP_E_UNSUPPORTED,
                        "%s: the batch plan needs %zu bytes, more than the fixed scratch holds (%zu); use apsp_batched",
                        who, need, kFixedScratchBytes - kWsAlign);
        base = ctx->fixed + kWsAlign;
    } else {
        if (!ctx->ws || ctx->ws_bytes < need)
            return fail(APSP_E_NOMEM, "%s needs a workspace of %zu bytes (have %zu; apsp_workspace_size)", who, need,
                        ctx->ws_bytes);
        base = ctx->ws;
    }
    auto* d_bptrs = reinterpret_cast<apsp::BatchPtrs*>(base);
    auto* d_ticket = reinterpret_cast<uint32_t*>(base + lay.ticket);
    auto* d_err = reinterpret_cast<uint32_t*>(base + lay.err);
    auto* d_qoff = reinterpret_cast<int32_t*>(base + lay.qoff);
    ctx->batch_err = d_err;
    auto* d_order = reinterpret_cast<int32_t*>(base + lay.order);
    auto* d_items = reinterpret_cast<int4*>(base + lay.items);
    auto* d_tasks = reinterpret_cast<apsp::BatchTask*>(base + lay.tasks);
    auto* d_counters = reinterpret_cast<int32_t*>(base + lay.counters);
    if (rebuild) {
        // the captured graphs (workspace path) belong to the previous plan;
        // they are dropped by the next call that would replay them
        ctx->border = std::move(order);
        ctx->litems = std::move(items);
        ctx->llaunches = std::move(launches);
        ctx->qtasks = std::move(qtasks);
        ctx->qoff = std::move(qoff);
        ctx->qcounters = qcounters;
        ctx->bkey = key;
        ctx->bcount = count;
        ctx->bdtype = dt;
        ctx->ws_owner = WS_NONE;
        ctx->fixed_serial = 0;
    }
    if (!pm.fixed && ctx->graph_key != ctx->bkey && (ctx->bexec || ctx->lexec || ctx->qexec)) {
        // a replay of the previous plan may still be running
        HIP_TRY(hipStreamSynchronize(st), "plan change sync");
        drop_batch_graphs(ctx);
    }
    if (!pm.fixed) ctx->graph_key = ctx->bkey;
    const bool resident = pm.fixed ? fixed_plan_resident(ctx) : ctx->ws_owner == WS_BATCHED;
    if (!resident) {
        // (re)upload the plan; the host vectors stay alive in the context, and
        // the stream is synchronised so that no later plan replaces them while
        // the copy may still read them (new batch shapes only)
        HIP_TRY(hipMemcpyAsync(d_order, ctx->border.data(), (size_t)count * sizeof(int32_t), hipMemcpyHostToDevice,
                               st),
                "plan upload");
        if (!ctx->litems.empty())
            HIP_TRY(hipMemcpyAsync(d_items, ctx->litems.data(), ctx->litems.size() * sizeof(int4),
                                   hipMemcpyHostToDevice, st),
                    "plan upload");
        if (!ctx->qtasks.empty())
            HIP_TRY(hipMemcpyAsync(d_tasks, ctx->qtasks.data(), ctx->qtasks.size() * sizeof(apsp::BatchTask),
                                   hipMemcpyHostToDevice, st),
                    "plan upload");
        if (!ctx->qoff.empty())
            HIP_TRY(hipMemcpyAsync(d_qoff, ctx->qoff.data(), ctx->qoff.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st),
                    "plan upload");
        HIP_TRY(apsp::launch_fill_u32(d_err, 0u, 1, st), "error word reset");
        HIP_TRY(hipStreamSynchronize(st), "plan upload sync");
        if (pm.fixed)
            fixed_plan_claim(ctx);
        else
            ctx->ws_owner = WS_BATCHED;
    }
    apsp::BatchArgs a{};
    a.data = data;
    a.offsets = d_offsets;
    a.sizes = d_sizes;
    a.order = d_order;
    a.count = count;
    a.counter = pm.fixed ? reinterpret_cast<uint32_t*>(ctx->fixed) : static_cast<uint32_t*>(ctx->d_scratch) + 8;
    const apsp::DType kdt = (apsp::DType)dt;
    const int grid = std::min<int>(count, ctx->num_cus * apsp::batched_resident_per_cu(kdt));
    const double terms = 0.0, bytes = 0.0;

    if ((o->flags & APSP_FLAG_BATCH_QUEUE) &&
        !(o->flags & (APSP_FLAG_BATCH_PERSISTENT | APSP_FLAG_BATCH_PER_GRAPH))) {
        // dependency-driven schedule: one workgroup per task, tickets in
        // topological order; zeroing the ticket and counters and the launch
        // are replayed from one captured graph per batch shape
        const int nx = (int)ctx->qoff.size() - 1;
        int qmax = 0;
        for (int x = 0; x < nx; ++x) qmax = std::max(qmax, ctx->qoff[x + 1] - ctx->qoff[x]);
        const int ncnt = ctx->qcounters;
        // one queue on a device of several XCDs: tasks release their tiles device-wide
        const bool global = nx == 1 && num_xcds(ctx) > 1;
        auto enqueue = [&](hipStream_t s2) -> hipError_t {
            return apsp::launch_batch_queue(kdt, d_bptrs, d_tasks, d_qoff, nx, qmax, d_ticket, d_counters, ncnt, d_err,
                                            global, s2);
        };
        return timed(ctx, APSP_KERNEL_OTHER, terms, bytes, st, [&]() -> apsp_status_t {
            HIP_TRY(apsp::launch_batch_ptrs(d_bptrs, data, d_offsets, d_sizes, st), "batch pointer update");
            if (pm.fixed || (o->flags & APSP_FLAG_BATCH_NO_GRAPH)) {
                HIP_TRY(enqueue(st), "queue launch");
                return APSP_OK;
            }
            if (!ctx->qexec) {
                HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal), "begin capture");
                hipError_t le = enqueue(ctx->capture);
                hipGraph_t g = nullptr;
                hipError_t ce = hipStreamEndCapture(ctx->capture, &g);
                if (le != hipSuccess) {
                    if (g) hipGraphDestroy(g);
                    return hip_fail(le, "queue capture launch");
                }
                HIP_TRY(ce, "end capture");
                hipGraphExec_t ex = nullptr;
                hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                if (ie != hipSuccess) {
                    hipGraphDestroy(g);
                    return hip_fail(ie, "graph instantiate");
                }
                ctx->qgraph = g;
                ctx->qexec = ex;
            }
            HIP_TRY(hipGraphLaunch(ctx->qexec, st), "graph launch");
            return APSP_OK;
        });
    }
    if (!(o->flags & (APSP_FLAG_BATCH_PERSISTENT | APSP_FLAG_BATCH_PER_GRAPH))) {
        // lock-step schedule: point the device record at this call's buffers,
        // then run the launch list (captured once per batch shape)
        auto enqueue = [&](hipStream_t s2) -> hipError_t {
            hipError_t e = hipSuccess;
            bool forked = false;
            auto join = [&]() -> hipError_t {
                hipError_t je = hipEventRecord(ctx->ev_p, ctx->side);
                if (je == hipSuccess) je = hipStreamWaitEvent(s2, ctx->ev_p, 0);
                forked = false;
                return je;
            };
            const bool two = ctx->side && ctx->ev_a && ctx->ev_p;
            for (const auto& L0 : ctx->llaunches) {
                apsp_ctx::Launch L = L0;
                L.side = L.side && two;
                if (L.side && !forked) {
                    // the side launches of round r start after its panels
                    if ((e = hipEventRecord(ctx->ev_a, s2)) != hipSuccess) return e;
                    if ((e = hipStreamWaitEvent(ctx->side, ctx->ev_a, 0)) != hipSuccess) return e;
                    forked = true;
                }
                if (!L.side && forked && L.phase == 1 && (e = join()) != hipSuccess) return e;
                e = apsp::launch_batch_phase(kdt, L.phase, d_bptrs, d_items + L.offset, L.count,
                                             L.side ? ctx->side : s2);
                if (e != hipSuccess) return e;
            }
            return forked ? join() : hipSuccess;
        };
        return timed(ctx, APSP_KERNEL_OTHER, terms, bytes, st, [&]() -> apsp_status_t {
            HIP_TRY(apsp::launch_batch_ptrs(d_bptrs, data, d_offsets, d_sizes, st), "batch pointer update");
            // a one-launch schedule (every graph n <= 128) runs faster as a
            // direct launch than as a graph replay
            if (pm.fixed || (o->flags & APSP_FLAG_BATCH_NO_GRAPH) || ctx->llaunches.size() <= 1) {
                HIP_TRY(enqueue(st), "lock-step launch");
                return APSP_OK;
            }
            if (!ctx->lexec) {
                HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal), "begin capture");
                hipError_t le = enqueue(ctx->capture);
                hipGraph_t g = nullptr;
                hipError_t ce = hipStreamEndCapture(ctx->capture, &g);
                if (le != hipSuccess) {
                    if (g) hipGraphDestroy(g);
                    return hip_fail(le, "lock-step capture launch");
                }
                HIP_TRY(ce, "end capture");
                hipGraphExec_t ex = nullptr;
                hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                if (ie != hipSuccess) {
                    hipGraphDestroy(g);
                    return hip_fail(ie, "graph instantiate");
                }
                ctx->lgraph = g;
                ctx->lexec = ex;
            }
            HIP_TRY(hipGraphLaunch(ctx->lexec, st), "graph launch");
            return APSP_OK;
        });
    }
    if (o->flags & APSP_FLAG_BATCH_PER_GRAPH) {
        // baseline: one launch (of the same kernel) per graph
        for (int32_t q = 0; q < count; ++q) {
            apsp::BatchArgs one = a;
            one.order = a.order + q;
            one.count = 1;
            rc = timed(ctx, APSP_KERNEL_OTHER, terms, bytes, st, [&]() -> apsp_status_t {
                HIP_TRY(apsp::launch_batched(kdt, one, 1, st), "per-graph launch");
                return APSP_OK;
            });
            if (rc) return rc;
        }
        return APSP_OK;
    }
    if (pm.fixed || (o->flags & APSP_FLAG_BATCH_NO_GRAPH)) {
        return timed(ctx, APSP_KERNEL_OTHER, terms, bytes, st, [&]() -> apsp_status_t {
            HIP_TRY(apsp::launch_batched(kdt, a, grid, st), "batched launch");
            return APSP_OK;
        });
    }
    if (!ctx->bexec) {
        // capture counter reset + persistent kernel once per batch shape
        HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t le = apsp::launch_batched(kdt, a, grid, ctx->capture);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(ctx->capture, &g);
        if (le != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(le, "batched capture launch");
        }
        HIP_TRY(ce, "end capture");
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            hipGraphDestroy(g);
            return hip_fail(ie, "graph instantiate");
        }
        size_t nn = 0;
        HIP_TRY(hipGraphGetNodes(g, nullptr, &nn), "graph nodes");
        std::vector<hipGraphNode_t> nodes(nn);
        HIP_TRY(hipGraphGetNodes(g, nodes.data(), &nn), "graph nodes");
        hipGraphNode_t kn = nullptr;
        hipKernelNodeParams kp{};
        for (hipGraphNode_t nd : nodes) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams q{};
            if (hipGraphKernelNodeGetParams(nd, &q) != hipSuccess) continue;
            if (q.func == apsp::batched_kernel(kdt)) {
                kn = nd;
                kp = q;
            }
        }
        if (!kn) {
            hipGraphExecDestroy(ex);
            hipGraphDestroy(g);
            return fail(APSP_E_HIP, "batched kernel node not found in the captured graph");
        }
        ctx->bgraph = g;
        ctx->bexec = ex;
        ctx->bnode = kn;
        ctx->bparams = kp;
        ctx->bargs = a;
    } else if (memcmp(&a, &ctx->bargs, sizeof a) != 0) {
        // same batch shape, new buffers: patch the kernel arguments in place
        hipKernelNodeParams kp = ctx->bparams;
        void* args[] = {&a};
        kp.kernelParams = args;
        kp.extra = nullptr;
        HIP_TRY(hipGraphExecKernelNodeSetParams(ctx->bexec, ctx->bnode, &kp), "graph node update");
        ctx->bargs = a;
    }
    return timed(ctx, APSP_KERNEL_OTHER, terms, bytes, st, [&]() -> apsp_status_t {
        HIP_TRY(hipGraphLaunch(ctx->bexec, st), "graph launch");
        return APSP_OK;
    });
}

}  // namespace

extern "C" {

apsp_status_t apsp_batched(apsp_ctx_t* ctx, apsp_dtype_t dt, int32_t count, void* data,
                           const int64_t* d_offsets, const int32_t* d_sizes, const int32_t* h_sizes,
                           const apsp_opts_t* opts, void* stream)
{
    return batched_common(ctx, dt, count, data, d_offsets, d_sizes, h_sizes, opts, stream, PlanMem{false},
                          "apsp_batched");
}

apsp_status_t apsp_batched_noalloc(apsp_ctx_t* ctx, apsp_dtype_t dt, int32_t count, void* data,
                                   const int64_t* d_offsets, const int32_t* d_sizes, const int32_t* h_sizes,
                                   const apsp_opts_t* opts, void* stream)
{
    return batched_common(ctx, dt, count, data, d_offsets, d_sizes, h_sizes, opts, stream, PlanMem{true},
                          "apsp_batched_noalloc");
}

apsp_status_t apsp_batched_status(apsp_ctx_t* ctx, void* stream, uint32_t* h_flags)
{
    apsp_status_t rc;
    if (!h_flags) return fail(APSP_E_ARG, "h_flags is NULL");
    if ((rc = check_ctx(ctx))) return rc;
    *h_flags = 0;
    if (!ctx->batch_err) return APSP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(h_flags, ctx->batch_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st), "status read");
    HIP_TRY(apsp::launch_fill_u32(ctx->batch_err, 0u, 1, st), "status reset");
    HIP_TRY(hipStreamSynchronize(st), "status sync");
    return APSP_OK;
}

apsp_status_t apsp_profile_enable(apsp_ctx_t* ctx, int32_t on)
{
    apsp_status_t rc;
    if ((rc = check_ctx(ctx))) return rc;
    for (const ProfRec& r : ctx->recs) {
        hipEventSynchronize(r.b);
    }
    ctx->recs.clear();
    ctx->pool_used = 0;
    ctx->prof = on != 0;
    ctx->prof_mask = (on == 1) ? 0xffffffffu : (uint32_t)on;
    return APSP_OK;
}

apsp_status_t apsp_profile_read(apsp_ctx_t* ctx, int32_t kind, apsp_kernel_stats_t* out)
{
    apsp_status_t rc;
    if (!out) return fail(APSP_E_ARG, "output is NULL");
    if (kind < 0 || kind >= APSP_KERNEL_KINDS) return fail(APSP_E_ARG, "kind = %d", kind);
    if ((rc = check_ctx(ctx))) return rc;
    *out = apsp_kernel_stats_t{};
    for (const ProfRec& r : ctx->recs) {
        if (r.kind != kind) continue;
        HIP_TRY(hipEventSynchronize(r.b), "profile event sync");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b), "profile elapsed");
        out->launches += 1;
        out->milliseconds += ms;
        out->terms += r.terms;
        out->bytes += r.bytes;
    }
    return APSP_OK;
}

int32_t apsp_candidate_count(void) { return kNumCandidates; }

apsp_status_t apsp_candidate(int32_t index, apsp_opts_t* out)
{
    if (!out) return fail(APSP_E_ARG, "output is NULL");
    if (index < 0 || index >= kNumCandidates) return fail(APSP_E_ARG, "candidate %d of %d", index, kNumCandidates);
    *out = apsp_opts_t{};
    const Candidate& c = kCandidates[index];
    out->algo = c.algo;
    out->block = c.block;
    out->tile = c.tile;
    out->closure = c.closure;
    out->cutover = c.cutover;
    out->flags = c.flags;
    return APSP_OK;
}

int32_t apsp_batch_candidate_count(void) { return kNumBatchCandidates; }

apsp_status_t apsp_batch_candidate(int32_t index, apsp_opts_t* out)
{
    if (!out) return fail(APSP_E_ARG, "output is NULL");
    if (index < 0 || index >= kNumBatchCandidates)
        return fail(APSP_E_ARG, "batch candidate %d of %d", index, kNumBatchCandidates);
    batch_candidate_opts(index, out);
    return APSP_OK;
}

apsp_status_t apsp_plan_batch(apsp_ctx_t* ctx, apsp_dtype_t dt, int32_t count, const int32_t* h_sizes,
                              double density, apsp_opts_t* out, int32_t* h_choice)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt))) return rc;
    if (!out) return fail(APSP_E_ARG, "output is NULL");
    if (count < 1 || !h_sizes || density < 0.0) return fail(APSP_E_ARG, "bad batch plan features");
    if ((rc = check_ctx(ctx))) return rc;
    int32_t choice = kDefaultBatchCandidate;
    if (h_choice) *h_choice = -1;
    int32_t max_n = 0;
    for (int32_t g = 0; g < count; ++g) max_n = std::max(max_n, h_sizes[g]);
    if (batch_model_ready(ctx)) {
        float x[4];
        batch_features(count, h_sizes, density, x);
        if ((rc = score_batch(ctx, x, max_n > apsp::batched_max_n(), nullptr, &choice))) return rc;
        if (h_choice) *h_choice = choice;
    }
    batch_candidate_opts(choice, out);
    // as apsp_batched's automatic plan: one queue for a batch of fewer graphs than XCDs
    if ((out->flags & APSP_FLAG_BATCH_QUEUE) && count < num_xcds(ctx)) out->flags |= APSP_FLAG_BATCH_GLOBAL;
    return APSP_OK;
}

apsp_status_t apsp_batched_choice(apsp_ctx_t* ctx, int32_t* h_choice)
{
    apsp_status_t rc;
    if (!h_choice) return fail(APSP_E_ARG, "h_choice is NULL");
    if ((rc = check_ctx(ctx))) return rc;
    *h_choice = ctx->bauto_choice;
    return APSP_OK;
}

apsp_status_t apsp_costmodel_init(apsp_ctx_t* ctx, int32_t K, uint64_t seed)
{
    apsp_status_t rc;
    if (K < 1 || K > 64) return fail(APSP_E_ARG, "K = %d (1..64)", K);
    if ((rc = check_ctx(ctx))) return rc;
    HIP_TRY(hipDeviceSynchronize(), "costmodel sync");
    free_costmodel(ctx);
    const int np = apsp::mlp_param_count(K);
    const size_t pb = (size_t)np * sizeof(float);
    const size_t wb = (size_t)apsp::mlp_workspace_floats(kCmMaxRows, K) * sizeof(float);
    hipError_t e = hipSuccess;
    for (auto pr : {std::make_pair(&ctx->cm_params, pb), std::make_pair(&ctx->cm_m, pb),
                    std::make_pair(&ctx->cm_v, pb), std::make_pair(&ctx->cm_grad, pb),
                    std::make_pair(&ctx->cm_ws, wb), std::make_pair(&ctx->cm_io, (size_t)(8 + K) * sizeof(float))})
        if (e == hipSuccess) e = hipMalloc(pr.first, pr.second);
    if (e != hipSuccess) {
        free_costmodel(ctx);
        return fail(APSP_E_NOMEM, "cost model allocation: %s", hipGetErrorString(e));
    }
    // He-uniform weights, zero biases
    std::vector<float> h(np, 0.f);
    const int H = apsp::kMlpHidden, I = apsp::kMlpIn;
    const int oW1 = 0, oW2 = I * H + H, oW3 = oW2 + H * H + H;
    auto fill = [&](int off, int count, int fan_in, uint64_t stream) {
        const double a = std::sqrt(6.0 / fan_in);
        const uint64_t key = mix64(seed + stream * 0x9E3779B97F4A7C15ull);
        for (int i = 0; i < count; ++i) {
            const double u = (double)(mix64(key + (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
            h[off + i] = (float)(a * (2.0 * u - 1.0));
        }
    };
    fill(oW1, I * H, I, 1);
    fill(oW2, H * H, H, 2);
    fill(oW3, H * K, H, 3);
    HIP_TRY(hipMemcpy(ctx->cm_params, h.data(), pb, hipMemcpyHostToDevice), "params upload");
    std::vector<float> z(np, 0.f);
    HIP_TRY(hipMemcpy(ctx->cm_m, z.data(), pb, hipMemcpyHostToDevice), "moment reset");
    HIP_TRY(hipMemcpy(ctx->cm_v, z.data(), pb, hipMemcpyHostToDevice), "moment reset");
    ctx->cm_K = K;
    ctx->cm_steps = 0;
    for (int i = 0; i < I; ++i) {
        ctx->cm_norm.mu[i] = 0.f;
        ctx->cm_norm.sd[i] = 1.f;
    }
    return APSP_OK;
}

apsp_status_t apsp_costmodel_set_norm(apsp_ctx_t* ctx, const float* mu, const float* sd)
{
    apsp_status_t rc;
    if (!mu || !sd) return fail(APSP_E_ARG, "NULL normalisation array");
    for (int i = 0; i < apsp::kMlpIn; ++i)
        if (!(sd[i] > 0.f)) return fail(APSP_E_ARG, "sd[%d] must be > 0", i);
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    for (int i = 0; i < apsp::kMlpIn; ++i) {
        ctx->cm_norm.mu[i] = mu[i];
        ctx->cm_norm.sd[i] = sd[i];
    }
    return APSP_OK;
}

apsp_status_t apsp_costmodel_set_params(apsp_ctx_t* ctx, const float* h, int64_t count)
{
    apsp_status_t rc;
    if (!h) return fail(APSP_E_ARG, "NULL parameter array");
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    const int np = apsp::mlp_param_count(ctx->cm_K);
    if (count != np) return fail(APSP_E_ARG, "count = %lld, model has %d parameters", (long long)count, np);
    HIP_TRY(hipDeviceSynchronize(), "costmodel sync");
    HIP_TRY(hipMemcpy(ctx->cm_params, h, (size_t)np * 4, hipMemcpyHostToDevice), "params upload");
    std::vector<float> z(np, 0.f);
    HIP_TRY(hipMemcpy(ctx->cm_m, z.data(), (size_t)np * 4, hipMemcpyHostToDevice), "moment reset");
    HIP_TRY(hipMemcpy(ctx->cm_v, z.data(), (size_t)np * 4, hipMemcpyHostToDevice), "moment reset");
    ctx->cm_steps = 0;
    return APSP_OK;
}

apsp_status_t apsp_costmodel_get_params(apsp_ctx_t* ctx, float* h, int64_t count)
{
    apsp_status_t rc;
    if (!h) return fail(APSP_E_ARG, "NULL parameter array");
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    const int np = apsp::mlp_param_count(ctx->cm_K);
    if (count != np) return fail(APSP_E_ARG, "count = %lld, model has %d parameters", (long long)count, np);
    HIP_TRY(hipDeviceSynchronize(), "costmodel sync");
    HIP_TRY(hipMemcpy(h, ctx->cm_params, (size_t)np * 4, hipMemcpyDeviceToHost), "params download");
    return APSP_OK;
}

apsp_status_t apsp_measure_fold_rate(apsp_ctx_t* ctx, int32_t fold, void* stream, double* h_terms_per_s,
                                     double* h_lane_instr_per_s)
{
    apsp_status_t rc;
    if (fold < APSP_FOLD_I32 || fold > APSP_FOLD_PACKED16) return fail(APSP_E_ARG, "fold = %d", fold);
    if (!h_terms_per_s || !h_lane_instr_per_s) return fail(APSP_E_ARG, "NULL output");
    if ((rc = check_ctx(ctx))) return rc;
    const apsp::DType dt = fold == APSP_FOLD_F32 ? apsp::F32 : fold == APSP_FOLD_PACKED16 ? apsp::I32P16 : apsp::I32;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = ctx->num_cus * 8;   // eight 4-wave workgroups per CU: 8 waves per SIMD
    const int iters = 65536;
    uint32_t* sink = static_cast<uint32_t*>(ctx->d_scratch) + 32;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = apsp::launch_fold_spin(dt, grid, iters / 16, 1u, sink, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = apsp::launch_fold_spin(dt, grid, iters, 2u, sink, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "fold-rate spin");
    if (!(ms > 0.f)) return fail(APSP_E_HIP, "fold-rate spin: no elapsed time");
    const apsp::FoldSpin f = apsp::fold_spin_shape(dt);
    const double lanes = (double)grid * apsp::fold_spin_threads() * iters;
    *h_terms_per_s = lanes * f.terms / (ms * 1e-3);
    *h_lane_instr_per_s = lanes * f.instr / (ms * 1e-3);
    return APSP_OK;
}

apsp_status_t apsp_costmodel_save(apsp_ctx_t* ctx, const char* path)
{
    apsp_status_t rc;
    if (!path) return fail(APSP_E_ARG, "NULL path");
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    const int K = ctx->cm_K;
    const int np = apsp::mlp_param_count(K);
    std::vector<float> h(np);
    HIP_TRY(hipDeviceSynchronize(), "costmodel sync");
    HIP_TRY(hipMemcpy(h.data(), ctx->cm_params, (size_t)np * 4, hipMemcpyDeviceToHost), "params download");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(APSP_E_ARG, "cannot open %s for writing", path);
    // %.9g prints every binary32 value so that it reads back exactly
    std::fprintf(f, "apsp-costmodel 1\nK %d\nin %d\nhidden %d\nmu", K, apsp::kMlpIn, apsp::kMlpHidden);
    for (int i = 0; i < apsp::kMlpIn; ++i) std::fprintf(f, " %.9g", (double)ctx->cm_norm.mu[i]);
    std::fprintf(f, "\nsd");
    for (int i = 0; i < apsp::kMlpIn; ++i) std::fprintf(f, " %.9g", (double)ctx->cm_norm.sd[i]);
    std::fprintf(f, "\nparams %d\n", np);
    for (int i = 0; i < np; ++i) std::fprintf(f, "%.9g\n", (double)h[i]);
    const bool ok = !std::ferror(f);
    if (std::fclose(f) != 0 || !ok) return fail(APSP_E_ARG, "writing %s failed", path);
    return APSP_OK;
}

apsp_status_t apsp_costmodel_load(apsp_ctx_t* ctx, const char* path)
{
    if (!path) return fail(APSP_E_ARG, "NULL path");
    // parse and check the whole file before touching the context
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(APSP_E_ARG, "cannot open %s", path);
    char tag[32] = {0};
    int ver = 0, K = 0, in = 0, hidden = 0, np = -1;
    float mu[apsp::kMlpIn], sd[apsp::kMlpIn];
    std::vector<float> h;
    const char* bad = nullptr;
    auto word = [&](const char* w) {
        char got[32] = {0};
        return std::fscanf(f, "%31s", got) == 1 && std::strcmp(got, w) == 0;
    };
    if (std::fscanf(f, "%31s %d", tag, &ver) != 2 || std::strcmp(tag, "apsp-costmodel") != 0 || ver != 1)
        bad = "header is not 'apsp-costmodel 1'";
    else if (!word("K") || std::fscanf(f, "%d", &K) != 1 || K < 1 || K > 64)
        bad = "K missing or outside 1..64";
    else if (!word("in") || std::fscanf(f, "%d", &in) != 1 || in != apsp::kMlpIn ||
             !word("hidden") || std::fscanf(f, "%d", &hidden) != 1 || hidden != apsp::kMlpHidden)
        bad = "layer sizes differ from this library's";
    if (!bad) {
        bool ok = word("mu");
        for (int i = 0; ok && i < apsp::kMlpIn; ++i) ok = std::fscanf(f, "%f", &mu[i]) == 1 && std::isfinite(mu[i]);
        ok = ok && word("sd");
        for (int i = 0; ok && i < apsp::kMlpIn; ++i) ok = std::fscanf(f, "%f", &sd[i]) == 1 && sd[i] > 0.f;
        if (!ok) bad = "mu / sd missing, not finite, or sd not positive";
    }
    if (!bad && (!word("params") || std::fscanf(f, "%d", &np) != 1 || np != apsp::mlp_param_count(K)))
        bad = "parameter count differs from the model size";
    if (!bad) {
        h.resize(np);
        for (int i = 0; i < np && !bad; ++i)
            if (std::fscanf(f, "%f", &h[i]) != 1 || !std::isfinite(h[i])) bad = "parameter missing or not finite";
    }
    std::fclose(f);
    if (bad) return fail(APSP_E_ARG, "%s: malformed cost model file (%s)", path, bad);
    apsp_status_t rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!ctx->cm_params || ctx->cm_K != K)
        if ((rc = apsp_costmodel_init(ctx, K, 0))) return rc;
    if ((rc = apsp_costmodel_set_norm(ctx, mu, sd))) return rc;
    return apsp_costmodel_set_params(ctx, h.data(), np);
}

apsp_status_t apsp_costmodel_train(apsp_ctx_t* ctx, const float* X, const float* T, const float* M, int32_t rows,
                                   const apsp_train_cfg_t* cfg, float* losses, void* stream)
{
    apsp_status_t rc;
    if (!X || !T || !M || !cfg) return fail(APSP_E_ARG, "NULL argument");
    if (rows < 1 || rows > kCmMaxRows) return fail(APSP_E_ARG, "rows = %d (1..%d)", rows, kCmMaxRows);
    if (cfg->steps < 1) return fail(APSP_E_ARG, "steps = %d", cfg->steps);
    if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
        !(cfg->eps > 0.f))
        return fail(APSP_E_ARG, "bad Adam hyper-parameters");
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    if (fault_injected("launch")) return fail(APSP_E_HIP, "injected launch failure");
    apsp::MlpAdam opt{cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, ctx->cm_steps};
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = timed(ctx, APSP_KERNEL_OTHER, 0.0, 0.0, st, [&]() -> apsp_status_t {
        HIP_TRY(apsp::launch_mlp_train(ctx->cm_params, ctx->cm_m, ctx->cm_v, ctx->cm_norm, X, T, M, rows, ctx->cm_K,
                                       cfg->steps, opt, ctx->cm_ws, ctx->cm_grad, losses, st),
                "mlp train launch");
        return APSP_OK;
    });
    if (rc == APSP_OK) ctx->cm_steps += cfg->steps;
    return rc;
}

apsp_status_t apsp_costmodel_grad(apsp_ctx_t* ctx, const float* X, const float* T, const float* M, int32_t rows,
                                  float* d_grad, float* d_loss, void* stream)
{
    apsp_status_t rc;
    if (!X || !T || !M || !d_grad) return fail(APSP_E_ARG, "NULL argument");
    if (rows < 1 || rows > kCmMaxRows) return fail(APSP_E_ARG, "rows = %d (1..%d)", rows, kCmMaxRows);
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    apsp::MlpAdam opt{1.f, 0.9f, 0.999f, 1e-8f, 0};
    HIP_TRY(apsp::launch_mlp_train(ctx->cm_params, ctx->cm_m, ctx->cm_v, ctx->cm_norm, X, T, M, rows, ctx->cm_K, 0,
                                   opt, ctx->cm_ws, d_grad, d_loss, st),
            "mlp grad launch");
    return APSP_OK;
}

apsp_status_t apsp_costmodel_forward(apsp_ctx_t* ctx, const float* X, int32_t rows, float* d_out, void* stream)
{
    apsp_status_t rc;
    if (!X || !d_out) return fail(APSP_E_ARG, "NULL argument");
    if (rows < 1 || rows > kCmMaxRows) return fail(APSP_E_ARG, "rows = %d (1..%d)", rows, kCmMaxRows);
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(apsp::launch_mlp_forward(ctx->cm_params, ctx->cm_norm, X, rows, ctx->cm_K, ctx->cm_ws, d_out, st),
            "mlp forward launch");
    return APSP_OK;
}

apsp_status_t apsp_costmodel_predict(apsp_ctx_t* ctx, const float* X, int32_t rows, int32_t* d_choice, void* stream)
{
    apsp_status_t rc;
    if (!X || !d_choice) return fail(APSP_E_ARG, "NULL argument");
    if (rows < 1 || rows > kCmMaxRows) return fail(APSP_E_ARG, "rows = %d (1..%d)", rows, kCmMaxRows);
    if ((rc = check_ctx(ctx)) || (rc = check_model(ctx))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // predictions land after the activations in the workspace
    float* out = ctx->cm_ws + apsp::mlp_workspace_floats(rows, ctx->cm_K) - (int64_t)rows * ctx->cm_K;
    HIP_TRY(apsp::launch_mlp_forward(ctx->cm_params, ctx->cm_norm, X, rows, ctx->cm_K, ctx->cm_ws, out, st),
            "mlp forward launch");
    HIP_TRY(apsp::launch_argmin_rows(out, rows, ctx->cm_K, d_choice, st), "argmin launch");
    return APSP_OK;
}

apsp_status_t apsp_plan(apsp_ctx_t* ctx, apsp_dtype_t dt, int64_t n, double density, int32_t batch,
                        int32_t connected, apsp_opts_t* out, int32_t* h_choice)
{
    apsp_status_t rc;
    if ((rc = check_dtype(dt))) return rc;
    if (!out) return fail(APSP_E_ARG, "output is NULL");
    if (n < 0 || batch < 1 || density < 0.0) return fail(APSP_E_ARG, "bad plan features");
    if (batch != 1) return fail(APSP_E_ARG, "apsp_plan plans one graph (batch = 1); use apsp_plan_batch");
    if ((rc = check_ctx(ctx))) return rc;
    if (h_choice) *h_choice = -1;
    if (!model_ready(ctx)) {
        *out = apsp_opts_t{};
        out->algo = n <= 4096 ? APSP_ALGO_FW : APSP_ALGO_RKLEENE;
        out->cutover = n <= 4096 ? 0 : 4096;
        return APSP_OK;
    }
    float x[4] = {(float)std::log2((double)std::max<int64_t>(n, 1)),
                  (float)std::log10(std::max(density, 1e-9)), (float)std::log2((double)batch),
                  connected ? 1.f : 0.f};
    HIP_TRY(hipMemcpy(ctx->cm_io, x, sizeof x, hipMemcpyHostToDevice), "plan features upload");
    if ((rc = apsp_costmodel_forward(ctx, ctx->cm_io, 1, ctx->cm_io + 4, nullptr))) return rc;
    std::vector<float> pred(ctx->cm_K);
    HIP_TRY(hipMemcpy(pred.data(), ctx->cm_io + 4, pred.size() * sizeof(float), hipMemcpyDeviceToHost),
            "plan scores download");
    // first minimum among the candidates this dtype can run
    const int32_t choice = pick_candidate(dt, pred.data());
    if (h_choice) *h_choice = choice;
    return apsp_candidate(choice, out);
}

}  // extern "C"
