// Min-plus (tropical) matrix product on the CDNA4 vector ALUs.
//
//   C[i][j] <- min(C[i][j], min_t A[i][t] (+) B[t][j])        (Sec. 3, Eq. 2)
//
// (min, +) is not a semiring the matrix cores implement, so the product runs
// on the VALUs.  Each workgroup owns an MT x NT output tile held in
// registers (TM x TN per lane); A and B slices of KT reduction steps are
// staged through LDS, double buffered, one barrier per slice.
//
// Reduction steps are consumed in pairs.  In LDS each element of a slice is
// stored as a pair (value at even t, value at odd t):
//   As[p][row] = (A[row][2p], A[row][2p+1]),   Bs[p][col] = (B[2p][col], B[2p+1][col]).
// int32: both halves are <= 2^30, so one 64-bit add (v_lshl_add_u64) forms
//        two terms without a carry crossing the halves, and one v_min3_u32
//        folds both into the accumulator: 2 instructions per 2 terms.
//        Saturation is free: sums stay <= 2^31 in u32 and the accumulator
//        starts at C <= INF, so min() never lets anything above INF through.
// fp32:  two v_add_f32 (one IEEE rounding each) and one v_min3_f32.
// int32, capped 16-bit mode: four steps per 64-bit LDS word, values capped at
//        14847 while staged; one 64-bit add and one v_pk_minimum3_f16 per
//        4 terms (SemP16).  Used by the solvers' PACKED16 option, which
//        checks the result and redoes the solve in int32 when any entry
//        reached the cap.
//
// Workgroup order: the flat grid is first redistributed so that consecutive
// tile indices land on the same XCD (the dispatcher deals workgroups to the
// 8 XCDs round-robin), then tiles are walked in groups of 8 tile rows so
// neighbouring workgroups share A rows and B columns in that XCD's L2.
#include "device.h"

#include <algorithm>

namespace apsp {

namespace {

using dev::Cfg;
using dev::SemF32;
using dev::SemI32;
using dev::SemP16;

template <class S, int MT, int NT, int KT, int TM, int TN, bool VEC, bool SKIP>
__global__ __launch_bounds__((MT / TM) * (NT / TN))
void k_minplus(const GemmGroup G, uint32_t* __restrict__ changed)
{
    using T = typename S::T;
    using P = typename S::P;
    __shared__ P As[2][KT / S::KPACK][MT + 2];
    __shared__ P Bs[2][KT / S::KPACK][NT + 2];

    // ---- which problem / split / tile this workgroup owns
    const int bid = dev::xcd_remap(blockIdx.x, gridDim.x);
    int pi = 0;
#pragma unroll
    for (int i = 1; i < kMaxGroup; ++i)
        if (i < G.count && bid >= G.p[i].wg_begin) pi = i;
    GemmProblem Pb = G.p[0];
#pragma unroll
    for (int i = 1; i < kMaxGroup; ++i)
        if (i == pi) Pb = G.p[i];

    const int local = bid - Pb.wg_begin;
    const int ntiles = Pb.tiles_m * Pb.tiles_n;
    if (ntiles <= 0) return;
    const int split = local / ntiles;
    const int t = local - split * ntiles;
    constexpr int GROUP = 8;
    const int group_w = GROUP * Pb.tiles_n;
    const int gidx = t / group_w;
    const int first_m = gidx * GROUP;
    const int gsz = min(Pb.tiles_m - first_m, GROUP);
    const int tin = t - gidx * group_w;
    int tm = first_m + tin % gsz;
    int tn = tin / gsz;
    if (Pb.skip_mc && tm >= Pb.skip_m0) tm += Pb.skip_mc;
    if (Pb.skip_nc && tn >= Pb.skip_n0) tn += Pb.skip_nc;
    const int kbeg = split * Pb.kchunk;
    const int kend = min(Pb.K, kbeg + Pb.kchunk);

    dev::mp_tile<S, MT, NT, KT, TM, TN, VEC, SKIP>(static_cast<const T*>(Pb.A), Pb.lda, static_cast<const T*>(Pb.B),
                                             Pb.ldb, static_cast<T*>(Pb.C), Pb.ldc, Pb.M, Pb.N, tm * MT, tn * NT,
                                             kbeg, kend, Pb.ksplit > 1, changed, As, Bs);
}

template <class S, int MT, int NT, int KT, int TM, int TN>
hipError_t launch_cfg(const GemmGroup& g, uint32_t* changed, bool skip, hipStream_t st)
{
    using C_ = Cfg<S, MT, NT, KT, TM, TN>;
    bool vec = true;
    for (int i = 0; i < g.count; ++i) {
        const GemmProblem& p = g.p[i];
        // vector accesses need element (4-byte) alignment only
        auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 3) == 0; };
        if (!al(p.A) || !al(p.B) || !al(p.C)) vec = false;
    }
    dim3 grid(g.total_wgs), block(C_::NTHR);
    if (skip) {
        if (vec)
            hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, true, true>), grid, block, 0, st, g, changed);
        else
            hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, false, true>), grid, block, 0, st, g, changed);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, true, false>), grid, block, 0, st, g, changed);
        else
            hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, false, false>), grid, block, 0, st, g, changed);
    }
    return hipGetLastError();
}

// Reduction slice per tile shape: 16 steps for 128-tiles, 32 for 64-tiles;
// the 16-bit mode (four steps per word) keeps 16 for 128-tiles, where its
// staging registers then stay few enough for three waves per SIMD, and
// takes 64 for 64-tiles.
template <class S>
hipError_t launch_sem(int tile, const GemmGroup& g, uint32_t* changed, bool skip, hipStream_t st)
{
    constexpr int X = S::KPACK / 2;
    if (tile == TILE_64) return launch_cfg<S, 64, 64, 32 * X, 4, 4>(g, changed, skip, st);
    return launch_cfg<S, 128, 128, 16, 8, 8>(g, changed, skip, st);
}

hipError_t launch_dtype(DType dt, int tile, const GemmGroup& g, uint32_t* changed, bool skip, hipStream_t st)
{
    if (dt == I32) return launch_sem<SemI32>(tile, g, changed, skip, st);
    if (dt == I32P16) return launch_sem<SemP16>(tile, g, changed, skip, st);
    return launch_sem<SemF32>(tile, g, changed, skip, st);
}

}  // namespace

TileShape tile_shape(int tile, DType dt)
{
    if (tile == TILE_64) return {64, 64, dt == I32P16 ? 64 : 32};
    return {128, 128, 16};
}

void finalize_group(GemmGroup& g, int tile, int split_target, DType dt)
{
    const TileShape ts = tile_shape(tile, dt);
    int64_t base_tiles = 0;
    for (int i = 0; i < g.count; ++i) {
        GemmProblem& p = g.p[i];
        const int fm = (p.M + ts.mt - 1) / ts.mt;
        const int fn = (p.N + ts.nt - 1) / ts.nt;
        p.tiles_m = std::max(0, fm - p.skip_mc);
        p.tiles_n = std::max(0, fn - p.skip_nc);
        base_tiles += (int64_t)p.tiles_m * p.tiles_n;
    }
    int32_t wg = 0;
    for (int i = 0; i < g.count; ++i) {
        GemmProblem& p = g.p[i];
        const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
        int ks = 1;
        if (split_target > 0 && tiles > 0 && base_tiles < split_target) {
            // enough reduction slices per split to amortise the prologue
            const int max_split = std::max(1, p.K / (4 * ts.kt));
            ks = (int)std::min<int64_t>(max_split, (split_target + base_tiles - 1) / base_tiles);
            ks = std::max(ks, 1);
        }
        int kchunk = p.K;
        if (ks > 1) {
            kchunk = (p.K + ks - 1) / ks;
            kchunk = (kchunk + ts.kt - 1) / ts.kt * ts.kt;
            ks = (p.K + kchunk - 1) / kchunk;
        }
        p.ksplit = ks;
        p.kchunk = std::max(kchunk, 1);
        p.wg_begin = wg;
        wg += (int32_t)(tiles * ks);
    }
    g.total_wgs = wg;
}

hipError_t launch_minplus(DType dt, int tile, const GemmGroup& g, bool skip, hipStream_t st)
{
    if (g.total_wgs <= 0) return hipSuccess;
    return launch_dtype(dt, tile, g, nullptr, skip, st);
}

hipError_t launch_square_pass(DType dt, int tile, void* D, int64_t n, int64_t ld,
                              uint32_t* d_changed, bool skip, hipStream_t st)
{
    GemmGroup g{};
    g.count = 1;
    GemmProblem& p = g.p[0];
    p.A = D; p.B = D; p.C = D;
    p.lda = p.ldb = p.ldc = ld;
    p.M = p.N = p.K = (int32_t)n;
    finalize_group(g, tile, 0, dt);
    if (g.total_wgs <= 0) return hipSuccess;
    return launch_dtype(dt, tile, g, d_changed, skip, st);
}

}  // namespace apsp
