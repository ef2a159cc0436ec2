// Cost-model MLP: x (4 features) -> Linear(4,64) + ReLU -> Linear(64,64) +
// ReLU -> Linear(64,K): one predicted (normalised) log run time per
// candidate plan; the planner takes the argmin.  Trained with masked mean
// squared error and Adam (Kingma & Ba 2015).
//
// Parameters are one flat fp32 array, row-major (input x output):
//   W1[4][64] | b1[64] | W2[64][64] | b2[64] | W3[64][K] | b3[K]
// Everything runs in a single workgroup: the model has ~5k parameters and the
// training sets a few hundred rows, so one workgroup that keeps every
// activation in a small global workspace is enough, and every sum is taken
// in a fixed order (no atomics): results are deterministic.
#include "internal.h"

namespace apsp {

namespace {

constexpr int H = 64;
constexpr int NT = 256;

struct Net {
    const float* W1;
    const float* b1;
    const float* W2;
    const float* b2;
    const float* W3;
    const float* b3;
};

__device__ __forceinline__ Net view(const float* p, int K)
{
    Net n;
    n.W1 = p;
    n.b1 = p + kMlpIn * H;
    n.W2 = n.b1 + H;
    n.b2 = n.W2 + H * H;
    n.W3 = n.b2 + H;
    n.b3 = n.W3 + H * K;
    (void)K;
    return n;
}

// Forward pass for rows [0, rows): Z1/H1/Z2/H2 (rows x 64) and OUT (rows x K).
__device__ void forward(const Net& w, const float* __restrict__ X, const MlpNorm& nm, int rows, int K,
                        float* Z1, float* H1, float* Z2, float* H2, float* OUT)
{
    for (int e = threadIdx.x; e < rows * H; e += NT) {
        const int r = e / H, u = e - r * H;
        float z = w.b1[u];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) z += ((X[r * kMlpIn + k] - nm.mu[k]) / nm.sd[k]) * w.W1[k * H + u];
        Z1[e] = z;
        H1[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * H; e += NT) {
        const int r = e / H, u = e - r * H;
        float z = w.b2[u];
        for (int k = 0; k < H; ++k) z += H1[r * H + k] * w.W2[k * H + u];
        Z2[e] = z;
        H2[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * K; e += NT) {
        const int r = e / K, c = e - r * K;
        float z = w.b3[c];
        for (int k = 0; k < H; ++k) z += H2[r * H + k] * w.W3[k * K + c];
        OUT[e] = z;
    }
    __syncthreads();
}

// Gradients of sum(mask * (out - T)^2) / max(1, sum(mask)) into G (flat,
// same layout as the parameters); returns the loss in *loss (thread 0).
__device__ void backward(const Net& w, const float* __restrict__ X, const MlpNorm& nm, const float* __restrict__ T,
                         const float* __restrict__ M, int rows, int K, const float* Z1, const float* H1,
                         const float* Z2, const float* H2, float* OUT, float* GZ2, float* GZ1, float* G,
                         float* red, float* loss)
{
    // mask count and loss, fixed-order block reduction
    float cnt = 0.f, l = 0.f;
    for (int e = threadIdx.x; e < rows * K; e += NT) {
        const float d = OUT[e] - T[e];
        cnt += M[e];
        l += M[e] * d * d;
    }
    red[threadIdx.x] = cnt;
    red[NT + threadIdx.x] = l;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x] += red[threadIdx.x + s];
            red[NT + threadIdx.x] += red[NT + threadIdx.x + s];
        }
        __syncthreads();
    }
    const float denom = red[0] > 1.f ? red[0] : 1.f;
    if (threadIdx.x == 0 && loss) *loss = red[NT] / denom;
    __syncthreads();
    // dL/dout, kept in OUT
    for (int e = threadIdx.x; e < rows * K; e += NT) OUT[e] = 2.f * (OUT[e] - T[e]) * M[e] / denom;
    __syncthreads();
    const int oW1 = 0, ob1 = kMlpIn * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H * K;
    // layer 3
    for (int e = threadIdx.x; e < H * K; e += NT) {
        const int k = e / K, c = e - k * K;
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += H2[r * H + k] * OUT[r * K + c];
        G[oW3 + e] = g;
    }
    for (int c = threadIdx.x; c < K; c += NT) {
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += OUT[r * K + c];
        G[ob3 + c] = g;
    }
    for (int e = threadIdx.x; e < rows * H; e += NT) {
        const int r = e / H, u = e - r * H;
        float g = 0.f;
        for (int c = 0; c < K; ++c) g += OUT[r * K + c] * w.W3[u * K + c];
        GZ2[e] = Z2[e] > 0.f ? g : 0.f;
    }
    __syncthreads();
    // layer 2
    for (int e = threadIdx.x; e < H * H; e += NT) {
        const int k = e / H, u = e - k * H;
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += H1[r * H + k] * GZ2[r * H + u];
        G[oW2 + e] = g;
    }
    for (int u = threadIdx.x; u < H; u += NT) {
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += GZ2[r * H + u];
        G[ob2 + u] = g;
    }
    for (int e = threadIdx.x; e < rows * H; e += NT) {
        const int r = e / H, k = e - r * H;
        float g = 0.f;
        for (int u = 0; u < H; ++u) g += GZ2[r * H + u] * w.W2[k * H + u];
        GZ1[e] = Z1[e] > 0.f ? g : 0.f;
    }
    __syncthreads();
    // layer 1
    for (int e = threadIdx.x; e < kMlpIn * H; e += NT) {
        const int k = e / H, u = e - k * H;
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += ((X[r * kMlpIn + k] - nm.mu[k]) / nm.sd[k]) * GZ1[r * H + u];
        G[oW1 + e] = g;
    }
    for (int u = threadIdx.x; u < H; u += NT) {
        float g = 0.f;
        for (int r = 0; r < rows; ++r) g += GZ1[r * H + u];
        G[ob1 + u] = g;
    }
    __syncthreads();
}

__global__ __launch_bounds__(NT) void k_mlp_forward(const float* __restrict__ P, MlpNorm nm,
                                                    const float* __restrict__ X, int rows, int K,
                                                    float* __restrict__ ws, float* __restrict__ out)
{
    const Net w = view(P, K);
    float* Z1 = ws;
    float* H1 = Z1 + rows * H;
    float* Z2 = H1 + rows * H;
    float* H2 = Z2 + rows * H;
    forward(w, X, nm, rows, K, Z1, H1, Z2, H2, out);
}

// steps == 0: one forward + backward, gradients left in G, no update.
// steps > 0: that many full-batch Adam steps; loss of every step in losses.
__global__ __launch_bounds__(NT) void k_mlp_train(float* __restrict__ P, float* __restrict__ Mo,
                                                  float* __restrict__ Vo, MlpNorm nm,
                                                  const float* __restrict__ X, const float* __restrict__ T,
                                                  const float* __restrict__ Msk, int rows, int K, int steps,
                                                  MlpAdam opt, float* __restrict__ ws, float* __restrict__ G,
                                                  float* __restrict__ losses)
{
    __shared__ float red[2 * NT];
    const int np = mlp_param_count(K);
    float* Z1 = ws;
    float* H1 = Z1 + rows * H;
    float* Z2 = H1 + rows * H;
    float* H2 = Z2 + rows * H;
    float* GZ2 = H2 + rows * H;
    float* GZ1 = GZ2 + rows * H;
    float* OUT = GZ1 + rows * H;
    const Net w = view(P, K);
    const int iters = steps > 0 ? steps : 1;
    float p1 = 1.f, p2 = 1.f;
    for (int s = 0; s < opt.t0; ++s) {
        p1 *= opt.beta1;
        p2 *= opt.beta2;
    }
    for (int it = 0; it < iters; ++it) {
        forward(w, X, nm, rows, K, Z1, H1, Z2, H2, OUT);
        backward(w, X, nm, T, Msk, rows, K, Z1, H1, Z2, H2, OUT, GZ2, GZ1, G, red, losses ? losses + it : nullptr);
        if (steps == 0) break;
        p1 *= opt.beta1;
        p2 *= opt.beta2;
        const float c1 = 1.f - p1, c2 = 1.f - p2;
        for (int e = threadIdx.x; e < np; e += NT) {
            const float g = G[e];
            const float m = opt.beta1 * Mo[e] + (1.f - opt.beta1) * g;
            const float v = opt.beta2 * Vo[e] + (1.f - opt.beta2) * g * g;
            Mo[e] = m;
            Vo[e] = v;
            P[e] -= opt.lr * (m / c1) / (sqrtf(v / c2) + opt.eps);
        }
        __syncthreads();
    }
}

__global__ void k_argmin_rows(const float* __restrict__ out, int rows, int K, int32_t* __restrict__ choice)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        int best = 0;
        float bv = out[r * K];
        for (int c = 1; c < K; ++c)
            if (out[r * K + c] < bv) {
                bv = out[r * K + c];
                best = c;
            }
        choice[r] = best;
    }
}

}  // namespace

hipError_t launch_mlp_forward(const float* P, const MlpNorm& nm, const float* X, int rows, int K, float* ws,
                              float* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_forward, dim3(1), dim3(NT), 0, st, P, nm, X, rows, K, ws, out);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float* P, float* M, float* V, const MlpNorm& nm, const float* X, const float* T,
                            const float* Msk, int rows, int K, int steps, const MlpAdam& opt, float* ws, float* G,
                            float* losses, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(NT), 0, st, P, M, V, nm, X, T, Msk, rows, K, steps, opt, ws, G,
                       losses);
    return hipGetLastError();
}

hipError_t launch_argmin_rows(const float* out, int rows, int K, int32_t* choice, hipStream_t st)
{
    const int blocks = (rows + 255) / 256;
    hipLaunchKernelGGL(k_argmin_rows, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, out, rows, K, choice);
    return hipGetLastError();
}

}  // namespace apsp
