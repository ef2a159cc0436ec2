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
//
// Workgroup order: the flat grid is first redistributed so that consecutive
// tile indices land on the same XCD (the dispatcher deals workgroups to the
// 8 XCDs round-robin), then tiles are walked in groups of 8 tile rows so
// neighbouring workgroups share A rows and B columns in that XCD's L2.
#include "internal.h"

#include <algorithm>

namespace apsp {

namespace {

struct SemI32 {
    using T = uint32_t;
    using P = uint64_t;
    static __device__ __forceinline__ T inf() { return kInfI32; }
    static __device__ __forceinline__ P pack(T lo, T hi) { return ((P)hi << 32) | (P)lo; }
    static __device__ __forceinline__ T fold(T acc, P a, P b) {
        P s = a + b;   // two independent 32-bit sums, no carry between halves
        // written as one three-input min so that the compiler cannot
        // re-associate consecutive steps into min(lo, hi) pairs (which
        // costs an extra instruction and a live register per accumulator)
        T r;
        asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"((T)s), "v"((T)(s >> 32)));
        return r;
    }
    static __device__ __forceinline__ void atomic_min(T* p, T v) { atomicMin(p, v); }
};

struct SemF32 {
    using T = float;
    using P = float2;
    static __device__ __forceinline__ T inf() { return __builtin_inff(); }
    static __device__ __forceinline__ P pack(T lo, T hi) { return make_float2(lo, hi); }
    static __device__ __forceinline__ T fold(T acc, P a, P b) {
        const T s0 = a.x + b.x, s1 = a.y + b.y;
        T r;
        asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(s0), "v"(s1));
        return r;
    }
    // Non-negative binary32 values order like their bit patterns read as
    // signed integers (+inf = 0x7f800000 is the largest), so an integer
    // atomic min is an exact float min here.
    static __device__ __forceinline__ void atomic_min(T* p, T v) {
        atomicMin(reinterpret_cast<int*>(p), __float_as_int(v));
    }
};

template <class P>
struct alignas(2 * sizeof(P)) Pair2 { P x, y; };

__device__ __forceinline__ int xcd_remap(int b, int G) {
    constexpr int X = 8;
    const int q = G / X, r = G % X;
    const int x = b % X, s = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

template <class S, int MT, int NT, int KT, int TM, int TN>
struct Cfg {
    static constexpr int TX = NT / TN;
    static constexpr int TY = MT / TM;
    static constexpr int NTHR = TX * TY;
    static constexpr int KP = KT / 2;
    static constexpr int GM = TM / 2;       // row groups of 2 per lane
    static constexpr int GN = TN / 2;
    static constexpr int SM = MT / GM;      // stride between a lane's row groups
    static constexpr int SN = NT / GN;
    static constexpr int PADP = 2;          // pairs of padding per LDS row
    static constexpr int LDA = MT + PADP;
    static constexpr int LDB = NT + PADP;
    // staging work per lane
    static constexpr int A_VECS = MT * KT / 4;          // float4-sized loads of A
    static constexpr int B_COMBOS = KP * (NT / 4);      // (pair row, 4 columns) of B
    static_assert(A_VECS % NTHR == 0, "A staging must divide evenly");
    static_assert(B_COMBOS % NTHR == 0, "B staging must divide evenly");
    static constexpr int A_PER = A_VECS / NTHR;
    static constexpr int B_PER = B_COMBOS / NTHR;
    static_assert(SM == 2 * TY && SN == 2 * TX, "lane row/col groups must tile the block");
};

template <class S, int MT, int NT, int KT, int TM, int TN, bool VEC>
__global__ __launch_bounds__((MT / TM) * (NT / TN))
void k_minplus(const GemmGroup G, uint32_t* __restrict__ changed)
{
    using C_ = Cfg<S, MT, NT, KT, TM, TN>;
    using T = typename S::T;
    using P = typename S::P;
    constexpr int KP = C_::KP;

    __shared__ P As[2][KP][C_::LDA];
    __shared__ P Bs[2][KP][C_::LDB];

    // ---- which problem / split / tile this workgroup owns
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
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
    const int m0 = tm * MT, n0 = tn * NT;
    const int kbeg = split * Pb.kchunk;
    const int kend = min(Pb.K, kbeg + Pb.kchunk);
    const bool atomic_out = Pb.ksplit > 1;

    const T* __restrict__ A = static_cast<const T*>(Pb.A);
    const T* __restrict__ B = static_cast<const T*>(Pb.B);
    T* C = static_cast<T*>(Pb.C);
    const int64_t lda = Pb.lda, ldb = Pb.ldb, ldc = Pb.ldc;
    const int M = Pb.M, N = Pb.N;

    const int tid = threadIdx.x;
    const int tx = tid % C_::TX;
    const int ty = tid / C_::TX;

    auto row_of = [&](int i) { return (i >> 1) * C_::SM + ty * 2 + (i & 1); };
    auto col_of = [&](int j) { return (j >> 1) * C_::SN + tx * 2 + (j & 1); };

    // ---- accumulators start at C (or INF for a partial-K split)
    T acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + row_of(i);
#pragma unroll
        for (int j = 0; j < TN; j += 2) {
            const int c = n0 + col_of(j);
            if (atomic_out) {
                acc[i][j] = S::inf();
                acc[i][j + 1] = S::inf();
            } else if (VEC && r < M && c + 1 < N) {
                const auto v = *reinterpret_cast<const Pair2<T>*>(C + (int64_t)r * ldc + c);
                acc[i][j] = v.x;
                acc[i][j + 1] = v.y;
            } else {
                acc[i][j] = (r < M && c < N) ? C[(int64_t)r * ldc + c] : S::inf();
                acc[i][j + 1] = (r < M && c + 1 < N) ? C[(int64_t)r * ldc + c + 1] : S::inf();
            }
        }
    }

    // ---- staging registers
    T ra[C_::A_PER][4];
    T rb[C_::B_PER][2][4];

    auto load_slice = [&](int k0) {
#pragma unroll
        for (int q = 0; q < C_::A_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const int row = L / (KT / 4);
            const int c4 = L % (KT / 4);
            const int gr = m0 + row;
            const int gk = k0 + c4 * 4;
            if (VEC && gr < M && gk + 3 < kend) {
                const float4 v = *reinterpret_cast<const float4*>(A + (int64_t)gr * lda + gk);
                ra[q][0] = __builtin_bit_cast(T, v.x);
                ra[q][1] = __builtin_bit_cast(T, v.y);
                ra[q][2] = __builtin_bit_cast(T, v.z);
                ra[q][3] = __builtin_bit_cast(T, v.w);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    ra[q][e] = (gr < M && gk + e < kend) ? A[(int64_t)gr * lda + gk + e] : S::inf();
            }
        }
#pragma unroll
        for (int q = 0; q < C_::B_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const int p = L / (NT / 4);
            const int c4 = L % (NT / 4);
            const int gc = n0 + c4 * 4;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int gk = k0 + 2 * p + h;
                if (VEC && gk < kend && gc + 3 < N) {
                    const float4 v = *reinterpret_cast<const float4*>(B + (int64_t)gk * ldb + gc);
                    rb[q][h][0] = __builtin_bit_cast(T, v.x);
                    rb[q][h][1] = __builtin_bit_cast(T, v.y);
                    rb[q][h][2] = __builtin_bit_cast(T, v.z);
                    rb[q][h][3] = __builtin_bit_cast(T, v.w);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[q][h][e] = (gk < kend && gc + e < N) ? B[(int64_t)gk * ldb + gc + e] : S::inf();
                }
            }
        }
    };

    auto store_slice = [&](int buf) {
#pragma unroll
        for (int q = 0; q < C_::A_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const int row = L / (KT / 4);
            const int c4 = L % (KT / 4);
            As[buf][c4 * 2][row] = S::pack(ra[q][0], ra[q][1]);
            As[buf][c4 * 2 + 1][row] = S::pack(ra[q][2], ra[q][3]);
        }
#pragma unroll
        for (int q = 0; q < C_::B_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const int p = L / (NT / 4);
            const int c4 = L % (NT / 4);
            Pair2<P> lo, hi;
            lo.x = S::pack(rb[q][0][0], rb[q][1][0]);
            lo.y = S::pack(rb[q][0][1], rb[q][1][1]);
            hi.x = S::pack(rb[q][0][2], rb[q][1][2]);
            hi.y = S::pack(rb[q][0][3], rb[q][1][3]);
            *reinterpret_cast<Pair2<P>*>(&Bs[buf][p][c4 * 4]) = lo;
            *reinterpret_cast<Pair2<P>*>(&Bs[buf][p][c4 * 4 + 2]) = hi;
        }
    };

    const int nslices = (kend > kbeg) ? (kend - kbeg + KT - 1) / KT : 0;
    if (nslices > 0) {
        load_slice(kbeg);
        store_slice(0);
        __syncthreads();
        for (int s = 0; s < nslices; ++s) {
            const int cur = s & 1;
            if (s + 1 < nslices) load_slice(kbeg + (s + 1) * KT);
            // two pair-steps per iteration: enough independent work to hide
            // LDS latency without hoisting every slice read into registers
#pragma unroll 2
            for (int p = 0; p < KP; ++p) {
                P a[TM], b[TN];
#pragma unroll
                for (int g = 0; g < C_::GM; ++g) {
                    const auto v = *reinterpret_cast<const Pair2<P>*>(&As[cur][p][g * C_::SM + ty * 2]);
                    a[2 * g] = v.x;
                    a[2 * g + 1] = v.y;
                }
#pragma unroll
                for (int g = 0; g < C_::GN; ++g) {
                    const auto v = *reinterpret_cast<const Pair2<P>*>(&Bs[cur][p][g * C_::SN + tx * 2]);
                    b[2 * g] = v.x;
                    b[2 * g + 1] = v.y;
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = S::fold(acc[i][j], a[i], b[j]);
            }
            if (s + 1 < nslices) store_slice(cur ^ 1);
            __syncthreads();
        }
    }

    // ---- epilogue
    bool dec = false;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + row_of(i);
#pragma unroll
        for (int j = 0; j < TN; j += 2) {
            const int c = n0 + col_of(j);
            if (atomic_out) {
                if (r < M && c < N && acc[i][j] < S::inf()) S::atomic_min(C + (int64_t)r * ldc + c, acc[i][j]);
                if (r < M && c + 1 < N && acc[i][j + 1] < S::inf())
                    S::atomic_min(C + (int64_t)r * ldc + c + 1, acc[i][j + 1]);
                continue;
            }
            if (changed) {
                // squaring pass: report whether this tile decreased anything
                if (r < M && c < N && acc[i][j] < C[(int64_t)r * ldc + c]) dec = true;
                if (r < M && c + 1 < N && acc[i][j + 1] < C[(int64_t)r * ldc + c + 1]) dec = true;
            }
            if (VEC && r < M && c + 1 < N) {
                Pair2<T> v;
                v.x = acc[i][j];
                v.y = acc[i][j + 1];
                *reinterpret_cast<Pair2<T>*>(C + (int64_t)r * ldc + c) = v;
            } else {
                if (r < M && c < N) C[(int64_t)r * ldc + c] = acc[i][j];
                if (r < M && c + 1 < N) C[(int64_t)r * ldc + c + 1] = acc[i][j + 1];
            }
        }
    }
    if (changed) {
        // one vector store per wave that saw a decrease
        if (__builtin_amdgcn_read_exec() && __any(dec) && (tid % warpSize) == 0) atomicOr(changed, 1u);
    }
}

template <class S, int MT, int NT, int KT, int TM, int TN>
hipError_t launch_cfg(const GemmGroup& g, uint32_t* changed, hipStream_t st)
{
    using C_ = Cfg<S, MT, NT, KT, TM, TN>;
    bool vec = true;
    for (int i = 0; i < g.count; ++i) {
        const GemmProblem& p = g.p[i];
        auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
        if ((p.lda & 3) || (p.ldb & 3) || (p.ldc & 3) || !al(p.A) || !al(p.B) || !al(p.C)) vec = false;
    }
    dim3 grid(g.total_wgs), block(C_::NTHR);
    if (vec)
        hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, true>), grid, block, 0, st, g, changed);
    else
        hipLaunchKernelGGL((k_minplus<S, MT, NT, KT, TM, TN, false>), grid, block, 0, st, g, changed);
    return hipGetLastError();
}

template <class S>
hipError_t launch_sem(int tile, const GemmGroup& g, uint32_t* changed, hipStream_t st)
{
    if (tile == TILE_64) return launch_cfg<S, 64, 64, 32, 4, 4>(g, changed, st);
    return launch_cfg<S, 128, 128, 16, 8, 8>(g, changed, st);
}

}  // namespace

TileShape tile_shape(int tile)
{
    if (tile == TILE_64) return {64, 64, 32};
    return {128, 128, 16};
}

void finalize_group(GemmGroup& g, int tile, int split_target)
{
    const TileShape ts = tile_shape(tile);
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

hipError_t launch_minplus(DType dt, int tile, const GemmGroup& g, hipStream_t st)
{
    if (g.total_wgs <= 0) return hipSuccess;
    if (dt == I32) return launch_sem<SemI32>(tile, g, nullptr, st);
    return launch_sem<SemF32>(tile, g, nullptr, st);
}

hipError_t launch_square_pass(DType dt, int tile, void* D, int64_t n, int64_t ld,
                              uint32_t* d_changed, hipStream_t st)
{
    GemmGroup g{};
    g.count = 1;
    GemmProblem& p = g.p[0];
    p.A = D; p.B = D; p.C = D;
    p.lda = p.ldb = p.ldc = ld;
    p.M = p.N = p.K = (int32_t)n;
    finalize_group(g, tile, 0);
    if (g.total_wgs <= 0) return hipSuccess;
    if (dt == I32) return launch_sem<SemI32>(tile, g, d_changed, st);
    return launch_sem<SemF32>(tile, g, d_changed, st);
}

}  // namespace apsp
