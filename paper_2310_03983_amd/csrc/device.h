// Device-side building blocks shared by the min-plus product, the tile
// closure and the batched kernel: element semantics, the register-blocked
// min-plus tile and the in-workgroup block closure.
#pragma once

#include "internal.h"

namespace apsp {
namespace dev {

constexpr int kMaxS = 128;   // largest block closed inside one workgroup

// A semiring policy gives: the element type T in memory, the packed LDS
// operand P holding KPACK consecutive reduction steps, the accumulator type
// A, and fold(acc, a, b) = min(acc, a_t + b_t over the KPACK steps).
// acc_from maps a C value to an accumulator, acc_value maps it back.
struct SemI32 {
    using T = uint32_t;
    using P = uint64_t;
    using A = uint32_t;
    static constexpr int KPACK = 2;
    static __device__ __forceinline__ T inf() { return kInfI32; }
    static __device__ __forceinline__ A acc_from(T c) { return c; }
    static __device__ __forceinline__ T acc_value(A a) { return a; }
    static __device__ __forceinline__ P pack(T lo, T hi) { return ((P)hi << 32) | (P)lo; }
    static __device__ __forceinline__ P pair(T lo, T hi) { return pack(lo, hi); }
    // one term: saturation is implicit (operands <= 2^30, accumulator <= INF)
    static __device__ __forceinline__ T relax(T x, T a, T b) { return min(x, a + b); }
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
    using A = float;
    static constexpr int KPACK = 2;
    static __device__ __forceinline__ T inf() { return __builtin_inff(); }
    static __device__ __forceinline__ A acc_from(T c) { return c; }
    static __device__ __forceinline__ T acc_value(A a) { return a; }
    static __device__ __forceinline__ P pack(T lo, T hi) { return make_float2(lo, hi); }
    static __device__ __forceinline__ P pair(T lo, T hi) { return pack(lo, hi); }
    static __device__ __forceinline__ T relax(T x, T a, T b) { return fminf(x, a + b); }
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

// int32 distances folded in capped 16-bit arithmetic.  Every value v is
// staged as the 16-bit pattern min(v, kCap16) + 0x400, kCap16 = 14847
// standing for "no path"; four consecutive reduction steps share one 64-bit
// LDS word.  One 64-bit add forms the four sums (each at most
// 2 kCap16 + 0x800 = 0x7bfe, so no carry crosses a lane) and one
// v_pk_minimum3_f16 folds them into an accumulator of two 16-bit partial
// minima (even / odd steps): 2 instructions per 4 terms.  The minimum is an
// fp16 one applied to integer patterns: every pattern lies in
// [0x400, 0x7bff], the positive normal binary16 numbers, whose order is the
// order of their bit patterns (the offset keeps subnormals, and any flushing
// of them, out of play).  Sums and accumulators carry the offset 0x800.
// Capping commutes with min and with addition of non-negative values,
//   min(a + b, cap) = min(min(a, cap) + min(b, cap), cap),
// so the folded value is exactly min(true value, kCap16).  acc_value widens a
// capped value to INF; the product's epilogue keeps the old C entry whenever
// that is smaller (a capped result says only "not below kCap16").
struct SemP16 {
    using T = uint32_t;
    using P = uint64_t;
    using A = uint32_t;
    static constexpr int KPACK = 4;
    static constexpr uint32_t kCap16 = apsp::kCap16;
    static constexpr uint32_t kOff = 0x400u;   // smallest positive normal binary16 pattern
    static __device__ __forceinline__ T inf() { return kInfI32; }
    static __device__ __forceinline__ uint32_t pattern(T v) { return min(v, kCap16) + kOff; }
    static __device__ __forceinline__ P quad(T x0, T x1, T x2, T x3) {
        const uint32_t lo = pattern(x0) | (pattern(x1) << 16);
        const uint32_t hi = pattern(x2) | (pattern(x3) << 16);
        return ((P)hi << 32) | (P)lo;
    }
    static __device__ __forceinline__ A acc_from(T c) { return (min(c, kCap16) + 2 * kOff) * 0x10001u; }
    static __device__ __forceinline__ T acc_value(A a) {
        const uint32_t r = min(a & 0xffffu, a >> 16) - 2 * kOff;
        return r < kCap16 ? r : kInfI32;
    }
    static __device__ __forceinline__ A fold(A acc, P a, P b) {
        const P s = a + b;
        A r;
        asm("v_pk_minimum3_f16 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"((uint32_t)s), "v"((uint32_t)(s >> 32)));
        return r;
    }
    static __device__ __forceinline__ void atomic_min(T* p, T v) { atomicMin(p, v); }
};

template <class P>
struct alignas(2 * sizeof(P)) Pair2 { P x, y; };

// Global-memory vector access that assumes only element (4-byte) alignment:
// rows of a matrix with a leading dimension that is not a multiple of 4 start
// at any 4-byte boundary.  The compiler still emits one dwordx4 / dwordx2
// access (multi-dword accesses need dword alignment only).
template <class V, class T>
__device__ __forceinline__ V ld_vec(const T* p)
{
    V v;
    __builtin_memcpy(&v, p, sizeof(V));
    return v;
}
template <class V, class T>
__device__ __forceinline__ void st_vec(T* p, const V& v)
{
    __builtin_memcpy(p, &v, sizeof(V));
}

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
    static constexpr int KP = KT / S::KPACK;   // packed reduction steps per slice
    static constexpr int GM = TM / 2;       // row groups of 2 per lane
    static constexpr int GN = TN / 2;
    static constexpr int SM = MT / GM;      // stride between a lane's row groups
    static constexpr int SN = NT / GN;
    static constexpr int PADP = 2;          // pairs of padding per LDS row
    static constexpr int LDA = MT + PADP;
    static constexpr int LDB = NT + PADP;
    // staging work per lane.  B is staged in (packed row, BV columns)
    // pieces: 4 columns, or 2 when four-step packing leaves too few packed
    // rows per slice to give every lane a 4-column piece
    static constexpr int A_VECS = MT * KT / 4;          // float4-sized loads of A
    static constexpr int BV = (KP * (NT / 4) < NTHR) ? 2 : 4;
    static constexpr int B_COMBOS = KP * (NT / BV);     // (packed row, BV columns) of B
    static_assert(A_VECS % NTHR == 0, "A staging must divide evenly");
    static_assert(B_COMBOS % NTHR == 0, "B staging must divide evenly");
    static constexpr int A_PER = A_VECS / NTHR;
    static constexpr int B_PER = B_COMBOS / NTHR;
    static_assert(SM == 2 * TY && SN == 2 * TX, "lane row/col groups must tile the block");
};


// ---------------------------------------------------------------------------
// One MT x NT output tile of C <- min(C, A (min,+) B) over reduction steps
// [kbeg, kend), computed by one workgroup of (MT/TM)*(NT/TN) lanes.  A, B and
// C already point at the (0, 0) element of their windows; m0/n0 are the tile
// origin.  With atomic_out the tile's partial minimum is merged into C with
// atomic min (split reduction); otherwise C is read once and written once.
// As/Bs: LDS staging of 2 x KT/KPACK x (MT+2) and 2 x KT/KPACK x (NT+2)
// packed words.
// ---------------------------------------------------------------------------
// SKIP: a slice whose staged A values, or whose staged B values, are all INF
// is not folded -- each of its terms is >= INF and the accumulator starts at
// C <= INF, so it could change nothing.  Lanes that stage a finite value
// write the slice's number into an LDS word per buffer and operand; after
// the barrier every lane reads the same words, so the choice is uniform, and
// a word written for slice s is never read for another slice (no reset).
template <class S, int MT, int NT, int KT, int TM, int TN, bool VEC, bool SKIP = false>
__device__ __forceinline__ void mp_tile(const typename S::T* __restrict__ A, int64_t lda,
                                        const typename S::T* __restrict__ B, int64_t ldb,
                                        typename S::T* C, int64_t ldc, int M, int N,
                                        int m0, int n0, int kbeg, int kend, bool atomic_out,
                                        uint32_t* __restrict__ changed,
                                        typename S::P (*As)[KT / S::KPACK][MT + 2],
                                        typename S::P (*Bs)[KT / S::KPACK][NT + 2])
{
    using C_ = Cfg<S, MT, NT, KT, TM, TN>;
    using T = typename S::T;
    using P = typename S::P;
    using Acc = typename S::A;
    constexpr int KPACK = S::KPACK;
    constexpr int KP = C_::KP;
    const int tid = threadIdx.x;
    const int tx = tid % C_::TX;
    const int ty = tid / C_::TX;

    auto row_of = [&](int i) { return (i >> 1) * C_::SM + ty * 2 + (i & 1); };
    auto col_of = [&](int j) { return (j >> 1) * C_::SN + tx * 2 + (j & 1); };

    // ---- accumulators start at C (or INF for a partial-K split)
    Acc acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + row_of(i);
#pragma unroll
        for (int j = 0; j < TN; j += 2) {
            const int c = n0 + col_of(j);
            if (atomic_out) {
                acc[i][j] = S::acc_from(S::inf());
                acc[i][j + 1] = S::acc_from(S::inf());
            } else if (VEC && r < M && c + 1 < N) {
                const auto v = ld_vec<Pair2<T>>(C + (int64_t)r * ldc + c);
                acc[i][j] = S::acc_from(v.x);
                acc[i][j + 1] = S::acc_from(v.y);
            } else {
                acc[i][j] = S::acc_from((r < M && c < N) ? C[(int64_t)r * ldc + c] : S::inf());
                acc[i][j + 1] = S::acc_from((r < M && c + 1 < N) ? C[(int64_t)r * ldc + c + 1] : S::inf());
            }
        }
    }

    // ---- staging registers
    T ra[C_::A_PER][4];
    constexpr int BV = C_::BV;
    T rb[C_::B_PER][KPACK][BV];

    // Per-lane parts of the staging addresses, formed once per tile: each
    // slice then adds only a uniform offset (k0 for A, (k0 + h) * ldb for
    // B), so no 64-bit multiply runs inside the slice loop.
    int64_t a_off[C_::A_PER];   // (m0 + row) * lda + 4 * c4
    int64_t b_off[C_::B_PER];   // KPACK * p * ldb + gc
#pragma unroll
    for (int q = 0; q < C_::A_PER; ++q) {
        const int L = tid + q * C_::NTHR;
        a_off[q] = (int64_t)(m0 + L / (KT / 4)) * lda + (L % (KT / 4)) * 4;
    }
#pragma unroll
    for (int q = 0; q < C_::B_PER; ++q) {
        const int L = tid + q * C_::NTHR;
        b_off[q] = (int64_t)(KPACK * (L / (NT / BV))) * ldb + n0 + (L % (NT / BV)) * BV;
    }
    // a tile wholly inside the window: full slices need no bounds checks
    const bool full_tile = m0 + MT <= M && n0 + NT <= N;

    auto load_slice = [&](int k0) {
        const T* As0 = A + k0;
        if (VEC && full_tile && k0 + KT <= kend) {
            // uniform branch: every lane loads whole vectors
#pragma unroll
            for (int q = 0; q < C_::A_PER; ++q) {
                const float4 v = ld_vec<float4>(As0 + a_off[q]);
                ra[q][0] = __builtin_bit_cast(T, v.x);
                ra[q][1] = __builtin_bit_cast(T, v.y);
                ra[q][2] = __builtin_bit_cast(T, v.z);
                ra[q][3] = __builtin_bit_cast(T, v.w);
            }
#pragma unroll
            for (int h = 0; h < KPACK; ++h) {
                const T* Bs0 = B + (int64_t)(k0 + h) * ldb;
#pragma unroll
                for (int q = 0; q < C_::B_PER; ++q) {
                    if constexpr (BV == 4) {
                        const float4 v = ld_vec<float4>(Bs0 + b_off[q]);
                        rb[q][h][0] = __builtin_bit_cast(T, v.x);
                        rb[q][h][1] = __builtin_bit_cast(T, v.y);
                        rb[q][h][2] = __builtin_bit_cast(T, v.z);
                        rb[q][h][3] = __builtin_bit_cast(T, v.w);
                    } else {
                        const Pair2<T> v = ld_vec<Pair2<T>>(Bs0 + b_off[q]);
                        rb[q][h][0] = v.x;
                        rb[q][h][1] = v.y;
                    }
                }
            }
            return;
        }
        // edge tiles and the last partial slice: every element checked
#pragma unroll
        for (int q = 0; q < C_::A_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const bool row_ok = m0 + L / (KT / 4) < M;
            const int gk = k0 + (L % (KT / 4)) * 4;
            const T* src = As0 + a_off[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) ra[q][e] = (row_ok && gk + e < kend) ? src[e] : S::inf();
        }
#pragma unroll
        for (int h = 0; h < KPACK; ++h) {
            const T* Bs0 = B + (int64_t)(k0 + h) * ldb;
#pragma unroll
            for (int q = 0; q < C_::B_PER; ++q) {
                const int L = tid + q * C_::NTHR;
                const int gk = k0 + KPACK * (L / (NT / BV)) + h;
                const int gc = n0 + (L % (NT / BV)) * BV;
                const T* src = Bs0 + b_off[q];
#pragma unroll
                for (int e = 0; e < BV; ++e) rb[q][h][e] = (gk < kend && gc + e < N) ? src[e] : S::inf();
            }
        }
    };

    auto store_slice = [&](int buf) {
#pragma unroll
        for (int q = 0; q < C_::A_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            const int row = L / (KT / 4);
            const int c4 = L % (KT / 4);
            if constexpr (KPACK == 2) {
                As[buf][c4 * 2][row] = S::pack(ra[q][0], ra[q][1]);
                As[buf][c4 * 2 + 1][row] = S::pack(ra[q][2], ra[q][3]);
            } else {
                As[buf][c4][row] = S::quad(ra[q][0], ra[q][1], ra[q][2], ra[q][3]);
            }
        }
#pragma unroll
        for (int q = 0; q < C_::B_PER; ++q) {
            const int L = tid + q * C_::NTHR;
            if constexpr (BV == 2) {
                const int p = L / (NT / 2);
                const int c2 = L % (NT / 2);
                Pair2<P> v;
                if constexpr (KPACK == 2) {
                    v.x = S::pack(rb[q][0][0], rb[q][1][0]);
                    v.y = S::pack(rb[q][0][1], rb[q][1][1]);
                } else {
                    v.x = S::quad(rb[q][0][0], rb[q][1][0], rb[q][2][0], rb[q][3][0]);
                    v.y = S::quad(rb[q][0][1], rb[q][1][1], rb[q][2][1], rb[q][3][1]);
                }
                *reinterpret_cast<Pair2<P>*>(&Bs[buf][p][c2 * 2]) = v;
            } else {
                const int p = L / (NT / 4);
                const int c4 = L % (NT / 4);
                Pair2<P> lo, hi;
                if constexpr (KPACK == 2) {
                    lo.x = S::pack(rb[q][0][0], rb[q][1][0]);
                    lo.y = S::pack(rb[q][0][1], rb[q][1][1]);
                    hi.x = S::pack(rb[q][0][2], rb[q][1][2]);
                    hi.y = S::pack(rb[q][0][3], rb[q][1][3]);
                } else {
                    lo.x = S::quad(rb[q][0][0], rb[q][1][0], rb[q][2][0], rb[q][3][0]);
                    lo.y = S::quad(rb[q][0][1], rb[q][1][1], rb[q][2][1], rb[q][3][1]);
                    hi.x = S::quad(rb[q][0][2], rb[q][1][2], rb[q][2][2], rb[q][3][2]);
                    hi.y = S::quad(rb[q][0][3], rb[q][1][3], rb[q][2][3], rb[q][3][3]);
                }
                *reinterpret_cast<Pair2<P>*>(&Bs[buf][p][c4 * 4]) = lo;
                *reinterpret_cast<Pair2<P>*>(&Bs[buf][p][c4 * 4 + 2]) = hi;
            }
        }
    };

    __shared__ int live[2][2];   // [buffer][A, B]: last slice with a finite staged value (SKIP)
    auto mark = [&](int buf, int sidx) {
        if constexpr (SKIP) {
            bool fa = false, fb = false;
#pragma unroll
            for (int q = 0; q < C_::A_PER; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) fa |= ra[q][e] < S::inf();
#pragma unroll
            for (int q = 0; q < C_::B_PER; ++q)
#pragma unroll
                for (int h = 0; h < KPACK; ++h)
#pragma unroll
                    for (int e = 0; e < BV; ++e) fb |= rb[q][h][e] < S::inf();
            // one lane per wave writes (same-address LDS writes serialise)
            const bool wa = __any(fa), wb = __any(fb);
            if ((tid & (warpSize - 1)) == 0) {
                if (wa) live[buf][0] = sidx;
                if (wb) live[buf][1] = sidx;
            }
        }
    };

    const int nslices = (kend > kbeg) ? (kend - kbeg + KT - 1) / KT : 0;
    if (nslices > 0) {
        load_slice(kbeg);
        store_slice(0);
        mark(0, 0);
        __syncthreads();
        for (int s = 0; s < nslices; ++s) {
            const int cur = s & 1;
            if (s + 1 < nslices) load_slice(kbeg + (s + 1) * KT);
            // two pair-steps per iteration: enough independent work to hide
            // LDS latency without hoisting every slice read into registers
            auto fold_slice = [&]() {
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
            };
            if constexpr (SKIP) {
                if (live[cur][0] == s && live[cur][1] == s) fold_slice();
            } else {
                fold_slice();
            }
            if (s + 1 < nslices) {
                store_slice(cur ^ 1);
                mark(cur ^ 1, s + 1);
            }
            __syncthreads();
        }
    }

    // ---- epilogue
    bool dec = false;
    if constexpr (KPACK == 4) {
        // capped accumulators: widen, then keep the old entry where it is
        // smaller (a capped value only says "not below the cap")
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int r = m0 + row_of(i);
#pragma unroll
            for (int j = 0; j < TN; j += 2) {
                const int c = n0 + col_of(j);
                const T v0 = S::acc_value(acc[i][j]), v1 = S::acc_value(acc[i][j + 1]);
                if (atomic_out) {
                    if (r < M && c < N && v0 < S::inf()) S::atomic_min(C + (int64_t)r * ldc + c, v0);
                    if (r < M && c + 1 < N && v1 < S::inf()) S::atomic_min(C + (int64_t)r * ldc + c + 1, v1);
                    continue;
                }
                if (VEC && r < M && c + 1 < N) {
                    Pair2<T> o = ld_vec<Pair2<T>>(C + (int64_t)r * ldc + c);
                    if (v0 < o.x || v1 < o.y) dec = true;
                    o.x = min(o.x, v0);
                    o.y = min(o.y, v1);
                    st_vec(C + (int64_t)r * ldc + c, o);
                } else {
                    if (r < M && c < N) {
                        const T o = C[(int64_t)r * ldc + c];
                        if (v0 < o) {
                            dec = true;
                            C[(int64_t)r * ldc + c] = v0;
                        }
                    }
                    if (r < M && c + 1 < N) {
                        const T o = C[(int64_t)r * ldc + c + 1];
                        if (v1 < o) {
                            dec = true;
                            C[(int64_t)r * ldc + c + 1] = v1;
                        }
                    }
                }
            }
        }
        if (changed && __builtin_amdgcn_read_exec() && __any(dec) && (tid % warpSize) == 0) atomicOr(changed, 1u);
        return;
    }
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
                st_vec(C + (int64_t)r * ldc + c, v);
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

// Blocked form of the Eq. 1 k-loop for one block of s <= 128, in one
// workgroup of 256 lanes.  Lane (ty, tx) owns the 8 x 8 elements at rows
// ty + 16*i and columns tx + 16*j and keeps them in registers for the whole
// call.  The k range is cut into four 32-wide bands; with this interleaving,
// band r is exactly register rows/columns {2r, 2r+1} of every lane, so every
// round has the same shape on every lane.  Only the current band is shared
// through LDS: its 32 rows (R) and its 32 columns (Cc), 34 KB in all.
//   0. owners publish band r's rows and columns;
//   1. pivot block (band x band): closed by min-plus squaring to a fixpoint
//      (each pass doubles the hop reach; the closure equals the Eq. 1
//      k-loop's), or in close_block_wide by the k-loop itself, two steps per
//      barrier over all lanes;
//   2. panels: band rows x other columns <- P* (min,+) row panel and other
//      rows x band columns <- column panel (min,+) P*, from the pre-update
//      panels, then written back to R / Cc;
//   3. remainder: other x other <- min(., column panel (min,+) row panel),
//      registers only.
// Phases 2 and 3 fold two k at a time with the packed add / min3 pair of the
// product kernel.  Entries outside the block are INF, so steps past its
// edge change nothing.
constexpr int kBand = 32;
constexpr int kLdR = kMaxS + 2;          // R: kBand rows of kMaxS (+2: even, staggered banks)
constexpr int kLdC = kBand + 2;          // Cc: kMaxS rows of kBand (+2)
constexpr int kCloseLdsWords = kBand * kLdR + kMaxS * kLdC;

template <class S>
__device__ __forceinline__ void close_block(typename S::T* __restrict__ D, int64_t ld, int s,
                                            typename S::T* lds)
{
    using T = typename S::T;
    using P = typename S::P;
    T* R = lds;                       // R[kk * kLdR + col]  = X[p0 + kk][col]
    T* Cc = lds + kBand * kLdR;       // Cc[row * kLdC + kk] = X[row][p0 + kk]
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;

    T x[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = ty + 16 * i;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = tx + 16 * j;
            x[i][j] = (r < s && c < s) ? D[(int64_t)r * ld + c] : S::inf();
        }
    }

    const int rounds = (s + kBand - 1) / kBand;
    // fully unrolled so that the band's register rows/columns are constants
#pragma unroll
    for (int rd = 0; rd < kMaxS / kBand; ++rd) {
        if (rd >= rounds) break;
        const int p0 = kBand * rd;
        const int i0 = 2 * rd;               // register rows/cols of band rd
        // ---- 0. publish band rows and columns
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 8; ++j) R[(ty + 16 * a) * kLdR + tx + 16 * j] = x[i0 + a][j];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int b = 0; b < 2; ++b) Cc[(ty + 16 * i) * kLdC + tx + 16 * b] = x[i][i0 + b];
        __syncthreads();
        // ---- 1. pivot block: min-plus squaring to a fixpoint (Sec. 3.2 at band
        //      scale) on R, which holds the whole pivot in its band columns.
        //      Each pass doubles the hop reach, so at most 6 passes change
        //      anything for 32 vertices; a pass that changes nothing ends it.
        //      Cc's copy of the pivot is refreshed afterwards.
        for (int pass = 0; pass < 8; ++pass) {
            T np[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) np[a][b] = x[i0 + a][i0 + b];
#pragma unroll 4
            for (int kk = 0; kk < kBand; kk += 2) {
                P pa[2], pb[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) pa[a] = *reinterpret_cast<const P*>(&R[(ty + 16 * a) * kLdR + p0 + kk]);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    pb[b] = S::pair(R[kk * kLdR + tx + 16 * (i0 + b)], R[(kk + 1) * kLdR + tx + 16 * (i0 + b)]);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) np[a][b] = S::fold(np[a][b], pa[a], pb[b]);
            }
            int changed = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) changed |= np[a][b] < x[i0 + a][i0 + b];
            __syncthreads();                 // every read of this pass is done
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    x[i0 + a][i0 + b] = np[a][b];
                    R[(ty + 16 * a) * kLdR + tx + 16 * (i0 + b)] = np[a][b];
                }
            if (!__syncthreads_or(changed)) break;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) Cc[(ty + 16 * (i0 + a)) * kLdC + tx + 16 * b] = x[i0 + a][i0 + b];
        __syncthreads();
        // ---- 2. panels (from the pre-update panel values)
        T nr[2][8], nc[8][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 8; ++j) nr[a][j] = x[i0 + a][j];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int b = 0; b < 2; ++b) nc[i][b] = x[i][i0 + b];
#pragma unroll 2
        for (int kk = 0; kk < kBand; kk += 2) {
            P pa[8], pb[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) pa[i] = *reinterpret_cast<const P*>(&Cc[(ty + 16 * i) * kLdC + kk]);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                pb[j] = S::pair(R[kk * kLdR + tx + 16 * j], R[(kk + 1) * kLdR + tx + 16 * j]);
            // row panel: P*[row][k..k+1] + R[k..k+1][col]
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 8; ++j) nr[a][j] = S::fold(nr[a][j], pa[i0 + a], pb[j]);
            // column panel: C[row][k..k+1] + P*[k..k+1][col]
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int b = 0; b < 2; ++b) nc[i][b] = S::fold(nc[i][b], pa[i], pb[i0 + b]);
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (j == i0 || j == i0 + 1) continue;
                x[i0 + a][j] = nr[a][j];
                R[(ty + 16 * a) * kLdR + tx + 16 * j] = nr[a][j];
            }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i == i0 || i == i0 + 1) continue;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                x[i][i0 + b] = nc[i][b];
                Cc[(ty + 16 * i) * kLdC + tx + 16 * b] = nc[i][b];
            }
        }
        __syncthreads();
        // ---- 3. remainder: other rows x other columns (registers only)
#pragma unroll 2
        for (int kk = 0; kk < kBand; kk += 2) {
            P pa[8], pb[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) pa[i] = *reinterpret_cast<const P*>(&Cc[(ty + 16 * i) * kLdC + kk]);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                pb[j] = S::pair(R[kk * kLdR + tx + 16 * j], R[(kk + 1) * kLdR + tx + 16 * j]);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (i == i0 || i == i0 + 1) continue;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (j == i0 || j == i0 + 1) continue;
                    x[i][j] = S::fold(x[i][j], pa[i], pb[j]);
                }
            }
        }
        __syncthreads();                     // R / Cc are republished next round
    }

#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = ty + 16 * i;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = tx + 16 * j;
            if (r < s && c < s) D[(int64_t)r * ld + c] = x[i][j];
        }
    }
}

// The same blocked closure for a workgroup of 512 lanes (two waves per SIMD,
// so one wave's LDS reads and barriers hide behind the other's folds).
// Lane (ty, tx), ty < 16, tx < 32, owns the 8 x 4 elements at rows ty + 16*i
// and columns tx + 32*j; band r is register rows {2r, 2r+1} and register
// column r of every lane.  Phases, LDS layout (R / Cc, 34 KB) and results
// are those of close_block; with half the elements per lane it needs 126
// VGPRs instead of 162 and closes a 128 x 128 block in about two thirds of
// the time.
constexpr int kCloseWideThreads = 512;

// Value of v in lane `lane` (0..63) of the calling lane's wave.
__device__ __forceinline__ uint32_t group_value(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(lane << 2, (int)v);
}
__device__ __forceinline__ float group_value(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(v)));
}

template <class S>
__device__ __forceinline__ void close_block_wide(typename S::T* __restrict__ D, int64_t ld, int s,
                                                 typename S::T* lds)
{
    using T = typename S::T;
    using P = typename S::P;
    T* R = lds;                       // R[kk * kLdR + col]  = X[p0 + kk][col]
    T* Cc = lds + kBand * kLdR;       // Cc[row * kLdC + kk] = X[row][p0 + kk]
    const int tid = threadIdx.x;
    const int tx = tid & 31, ty = tid >> 5;

    T x[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = ty + 16 * i;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = tx + 32 * j;
            x[i][j] = (r < s && c < s) ? D[(int64_t)r * ld + c] : S::inf();
        }
    }

    const int rounds = (s + kBand - 1) / kBand;
#pragma unroll
    for (int rd = 0; rd < kMaxS / kBand; ++rd) {
        if (rd >= rounds) break;
        const int p0 = kBand * rd;
        const int i0 = 2 * rd;        // band rows are register rows i0, i0 + 1; band column is rd
        // ---- 0. publish the band
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) R[(ty + 16 * a) * kLdR + tx + 32 * j] = x[i0 + a][j];
#pragma unroll
        for (int i = 0; i < 8; ++i) Cc[(ty + 16 * i) * kLdC + tx] = x[i][rd];
        __syncthreads();
        // ---- 1. pivot block: the k-loop of Eq. 1 over the band's 32 steps,
        //      two steps per barrier.  Lane t holds entries (t / 16,
        //      2 (t % 16) + {0, 1}), so each 16-lane group holds one pivot row
        //      and its lane k / 2 holds the row's columns k and k + 1.  Steps
        //      k, k + 1 read rows k and k + 1 from R (their owners publish them
        //      after the previous pair); every lane applies step k to row
        //      k + 1 and to its own column k + 1 itself, then folds both
        //      steps: min(x, x_k + r_k, x'_{k+1} + r'_{k+1}).  Row k does not
        //      change in step k, nor column k.
        {
            const int pr = tid >> 4, pc = 2 * (tid & 15);
            T pv[2] = {R[pr * kLdR + p0 + pc], R[pr * kLdR + p0 + pc + 1]};
#pragma unroll
            for (int k = 0; k < kBand; k += 2) {
                const int src = (tid & 48) | (k >> 1);   // lane of the wave holding (pr, k), (pr, k + 1)
                const T c0 = group_value(pv[0], src), c1 = group_value(pv[1], src);
                const T* rk = R + k * kLdR + p0;
                const T* rk1 = rk + kLdR;
                const T a0 = rk[pc], a1 = rk[pc + 1];
                const T e0 = S::relax(rk1[pc], rk1[k], a0), e1 = S::relax(rk1[pc + 1], rk1[k], a1);
                const P ca = S::pair(c0, S::relax(c1, c0, rk[k + 1]));
                pv[0] = S::fold(pv[0], ca, S::pair(a0, e0));
                pv[1] = S::fold(pv[1], ca, S::pair(a1, e1));
                if ((pr >> 1) == (k >> 1) + 1) {   // rows k + 2, k + 3: read by the next pair
                    R[pr * kLdR + p0 + pc] = pv[0];
                    R[pr * kLdR + p0 + pc + 1] = pv[1];
                }
                __syncthreads();
            }
            R[pr * kLdR + p0 + pc] = pv[0];   // every row changes after it was published
            R[pr * kLdR + p0 + pc + 1] = pv[1];
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            x[i0 + a][rd] = R[(ty + 16 * a) * kLdR + p0 + tx];
            Cc[(ty + 16 * (i0 + a)) * kLdC + tx] = x[i0 + a][rd];
        }
        __syncthreads();
        // ---- 2. panels, from the closed pivot and the pre-update panels
        T nr[2][4], nc[8];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) nr[a][j] = x[i0 + a][j];
#pragma unroll
        for (int i = 0; i < 8; ++i) nc[i] = x[i][rd];
#pragma unroll 2
        for (int kk = 0; kk < kBand; kk += 2) {
            P pa[8], pb[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) pa[i] = *reinterpret_cast<const P*>(&Cc[(ty + 16 * i) * kLdC + kk]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                pb[j] = S::pair(R[kk * kLdR + tx + 32 * j], R[(kk + 1) * kLdR + tx + 32 * j]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 4; ++j) nr[a][j] = S::fold(nr[a][j], pa[i0 + a], pb[j]);
#pragma unroll
            for (int i = 0; i < 8; ++i) nc[i] = S::fold(nc[i], pa[i], pb[rd]);
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j == rd) continue;
                x[i0 + a][j] = nr[a][j];
                R[(ty + 16 * a) * kLdR + tx + 32 * j] = nr[a][j];
            }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i == i0 || i == i0 + 1) continue;
            x[i][rd] = nc[i];
            Cc[(ty + 16 * i) * kLdC + tx] = nc[i];
        }
        __syncthreads();
        // ---- 3. remainder: other rows x other columns (registers only)
#pragma unroll 2
        for (int kk = 0; kk < kBand; kk += 2) {
            P pa[8], pb[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) pa[i] = *reinterpret_cast<const P*>(&Cc[(ty + 16 * i) * kLdC + kk]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                pb[j] = S::pair(R[kk * kLdR + tx + 32 * j], R[(kk + 1) * kLdR + tx + 32 * j]);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (i == i0 || i == i0 + 1) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j == rd) continue;
                    x[i][j] = S::fold(x[i][j], pa[i], pb[j]);
                }
            }
        }
        __syncthreads();                     // R / Cc are republished next round
    }

#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = ty + 16 * i;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = tx + 32 * j;
            if (r < s && c < s) D[(int64_t)r * ld + c] = x[i][j];
        }
    }
}

}  // namespace dev
}  // namespace apsp
