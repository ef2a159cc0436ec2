// Last-hop predecessors (Sec. 2: pred[i][j] is the vertex before j on an
// i -> j path; Sec. 3.1 takes them from an argmin over the intermediate
// index).  Given distances D and costs W:
//
//   P[i][j] = the smallest v != j minimising D[i][v] (+) W[v][j],
//             or -1 when i == j or that minimum is not below INF.
//
// This is one min-plus product D (min,+) W' (W' = W with its diagonal set to
// INF) that also keeps the index of the minimum.  The index forbids the
// packed two-term fold of the distance kernels: every term is an add, a
// compare and two selects.  64 x 64 output tile per workgroup of 256 lanes
// (4 x 4 per lane), reduction staged through LDS in slices of 32; the
// reduction index runs in increasing order with a strict compare, so ties
// keep the smallest v.
#include "device.h"

namespace apsp {

namespace {

constexpr int MT = 64, NT = 64, KT = 32, TM = 4, TN = 4;

template <class S>
__global__ __launch_bounds__(256) void k_predecessors(const typename S::T* __restrict__ D, int64_t ldd,
                                                      const typename S::T* __restrict__ W, int64_t ldw,
                                                      int32_t* __restrict__ P, int64_t ldp, int n)
{
    using T = typename S::T;
    __shared__ T As[KT][MT + 1];   // As[k][row] = D[m0 + row][k0 + k]
    __shared__ T Bs[KT][NT + 1];   // Bs[k][col] = W[k0 + k][n0 + col] (INF on the diagonal)
    const int tiles_n = (n + NT - 1) / NT;
    const int bid = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int m0 = (bid / tiles_n) * MT, n0 = (bid % tiles_n) * NT;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;

    T acc[TM][TN];
    int32_t arg[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            acc[i][j] = S::inf();
            arg[i][j] = -1;
        }

    for (int k0 = 0; k0 < n; k0 += KT) {
        for (int e = tid; e < MT * KT; e += 256) {
            const int row = e / KT, k = e % KT;
            const int gr = m0 + row, gk = k0 + k;
            As[k][row] = (gr < n && gk < n) ? D[(int64_t)gr * ldd + gk] : S::inf();
        }
        for (int e = tid; e < KT * NT; e += 256) {
            const int k = e / NT, col = e % NT;
            const int gk = k0 + k, gc = n0 + col;
            Bs[k][col] = (gk < n && gc < n && gk != gc) ? W[(int64_t)gk * ldw + gc] : S::inf();
        }
        __syncthreads();
        for (int k = 0; k < KT; ++k) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const T s = a[i] + b[j];          // int32: <= 2^31, no wrap
                    if (s < acc[i][j]) {
                        acc[i][j] = s;
                        arg[i][j] = k0 + k;
                    }
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + ty + 16 * i;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int c = n0 + tx + 16 * j;
            if (r < n && c < n) P[(int64_t)r * ldp + c] = (r == c || !(acc[i][j] < S::inf())) ? -1 : arg[i][j];
        }
    }
}

}  // namespace

hipError_t launch_predecessors(DType dt, const void* D, int64_t ldd, const void* W, int64_t ldw, int32_t* P,
                               int64_t ldp, int32_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (int64_t)((n + MT - 1) / MT) * ((n + NT - 1) / NT);
    if (dt == I32)
        hipLaunchKernelGGL(k_predecessors<dev::SemI32>, dim3((unsigned)tiles), dim3(256), 0, st,
                           (const uint32_t*)D, ldd, (const uint32_t*)W, ldw, P, ldp, n);
    else
        hipLaunchKernelGGL(k_predecessors<dev::SemF32>, dim3((unsigned)tiles), dim3(256), 0, st,
                           (const float*)D, ldd, (const float*)W, ldw, P, ldp, n);
    return hipGetLastError();
}

}  // namespace apsp
