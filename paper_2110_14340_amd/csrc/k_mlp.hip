// FP32 kernels of the learned cost model (3 hidden layers of width 64,
// ReLU, scalar output) for gfx950: forward, backward, gradient reduction and
// Adam.  The network predicts the log run time of a loop nest under a launch
// configuration from a standardised feature vector.
//
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3)
//   yhat = w4 . h3 + b4 ;  L = mean_b (yhat_b - y_b)^2 ;  relu'(0) = 0
//
// Parameter vector layout (floats): W1 [64 x F] | b1 [64] | W2 [64 x 64] |
// b2 | W3 [64 x 64] | b3 | w4 [64] | b4 [1].  Weights are staged in LDS
// (about 37 KB for F = 12); one lane evaluates one sample, so every lane
// reads the same weight at the same time (LDS broadcast).  Gradients are
// reduced over the batch by one lane per parameter summing samples in
// increasing order (deterministic, no atomics).
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int H = kMlpHidden;

struct Off {
    int W1, b1, W2, b2, W3, b3, w4, b4, P;
};

__host__ __device__ inline Off offsets(int F) {
    Off o;
    o.W1 = 0;
    o.b1 = o.W1 + H * F;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + H * H;
    o.w4 = o.b3 + H;
    o.b4 = o.w4 + H;
    o.P = o.b4 + 1;
    return o;
}

constexpr int kMlpThreads = 128;

// Forward pass for samples [0, n): stores the standardised input, the three
// hidden activations (for the backward pass) and yhat.  idx (optional) maps
// sample b to row idx[b] of X.
__global__ void __launch_bounds__(kMlpThreads)
mlp_forward_kernel(const float *__restrict__ params, const float *__restrict__ mu, const float *__restrict__ sd,
                   const float *__restrict__ X, const int *__restrict__ idx, int n, int F, float *__restrict__ xs,
                   float *__restrict__ h1s, float *__restrict__ h2s, float *__restrict__ h3s,
                   float *__restrict__ yhat) {
    extern __shared__ float w[];
    const Off o = offsets(F);
    for (int i = threadIdx.x; i < o.P; i += blockDim.x) w[i] = params[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int row = idx ? idx[b] : b;
    // fixed-size register arrays: every index below is a compile-time
    // constant after unrolling, so nothing spills to scratch
    float x[kMlpMaxFeatures];
#pragma unroll
    for (int f = 0; f < kMlpMaxFeatures; ++f) {
        x[f] = 0.f;
        if (f < F) {
            x[f] = (X[(int64_t)row * F + f] - mu[f]) / sd[f];
            if (xs) xs[(int64_t)b * F + f] = x[f];
        }
    }
    float h1[H], h2[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float z = w[o.b1 + i];
#pragma unroll
        for (int f = 0; f < kMlpMaxFeatures; ++f)
            if (f < F) z += w[o.W1 + i * F + f] * x[f];
        h1[i] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float z = w[o.b2 + i];
#pragma unroll
        for (int j = 0; j < H; ++j) z += w[o.W2 + i * H + j] * h1[j];
        h2[i] = z > 0.f ? z : 0.f;
    }
    float y = w[o.b4];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float z = w[o.b3 + i];
#pragma unroll
        for (int j = 0; j < H; ++j) z += w[o.W3 + i * H + j] * h2[j];
        const float h3 = z > 0.f ? z : 0.f;
        if (h3s) h3s[(int64_t)b * H + i] = h3;
        y += w[o.w4 + i] * h3;
    }
    if (h1s) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            h1s[(int64_t)b * H + i] = h1[i];
            h2s[(int64_t)b * H + i] = h2[i];
        }
    }
    yhat[b] = y;
}

// Backward deltas per sample: g = 2 (yhat - y)/n; d3 = g w4 [h3>0];
// d2 = W3^T d3 [h2>0]; d1 = W2^T d2 [h1>0]; also the squared error.
__global__ void __launch_bounds__(kMlpThreads)
mlp_delta_kernel(const float *__restrict__ params, int F, const float *__restrict__ y, const int *__restrict__ idx,
                 int n, const float *__restrict__ yhat, const float *__restrict__ h1s, const float *__restrict__ h2s,
                 const float *__restrict__ h3s, float *__restrict__ g, float *__restrict__ d1s,
                 float *__restrict__ d2s, float *__restrict__ d3s, float *__restrict__ sqerr) {
    extern __shared__ float w[];
    const Off o = offsets(F);
    for (int i = threadIdx.x; i < o.P; i += blockDim.x) w[i] = params[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int row = idx ? idx[b] : b;
    const float e = yhat[b] - y[row];
    sqerr[b] = e * e;
    const float gb = 2.f * e / (float)n;
    g[b] = gb;
    float d3[H], d2[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        d3[i] = h3s[(int64_t)b * H + i] > 0.f ? gb * w[o.w4 + i] : 0.f;
        d3s[(int64_t)b * H + i] = d3[i];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) s += w[o.W3 + i * H + j] * d3[i];
        d2[j] = h2s[(int64_t)b * H + j] > 0.f ? s : 0.f;
        d2s[(int64_t)b * H + j] = d2[j];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) s += w[o.W2 + i * H + j] * d2[i];
        d1s[(int64_t)b * H + j] = h1s[(int64_t)b * H + j] > 0.f ? s : 0.f;
    }
}

// One lane per parameter: its gradient summed over samples b = 0..n-1.
__global__ void __launch_bounds__(256)
mlp_grad_kernel(int F, int n, const float *__restrict__ xs, const float *__restrict__ h1s,
                const float *__restrict__ h2s, const float *__restrict__ h3s, const float *__restrict__ g,
                const float *__restrict__ d1s, const float *__restrict__ d2s, const float *__restrict__ d3s,
                float *__restrict__ grad) {
    const Off o = offsets(F);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= o.P) return;
    float s = 0.f;
    if (k < o.b1) {  // W1[i][f] = sum d1[b][i] x[b][f]
        const int i = k / F, f = k % F;
        for (int b = 0; b < n; ++b) s += d1s[(int64_t)b * H + i] * xs[(int64_t)b * F + f];
    } else if (k < o.W2) {
        const int i = k - o.b1;
        for (int b = 0; b < n; ++b) s += d1s[(int64_t)b * H + i];
    } else if (k < o.b2) {
        const int i = (k - o.W2) / H, j = (k - o.W2) % H;
        for (int b = 0; b < n; ++b) s += d2s[(int64_t)b * H + i] * h1s[(int64_t)b * H + j];
    } else if (k < o.W3) {
        const int i = k - o.b2;
        for (int b = 0; b < n; ++b) s += d2s[(int64_t)b * H + i];
    } else if (k < o.b3) {
        const int i = (k - o.W3) / H, j = (k - o.W3) % H;
        for (int b = 0; b < n; ++b) s += d3s[(int64_t)b * H + i] * h2s[(int64_t)b * H + j];
    } else if (k < o.w4) {
        const int i = k - o.b3;
        for (int b = 0; b < n; ++b) s += d3s[(int64_t)b * H + i];
    } else if (k < o.b4) {
        const int j = k - o.w4;
        for (int b = 0; b < n; ++b) s += g[b] * h3s[(int64_t)b * H + j];
    } else {
        for (int b = 0; b < n; ++b) s += g[b];
    }
    grad[k] = s;
}

// Adam with bias correction, step t (1-based).
__global__ void __launch_bounds__(256)
mlp_adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ grad,
                int P, int t, float lr, float beta1, float beta2, float eps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const float gk = grad[k];
    const float mk = beta1 * m[k] + (1.f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float c1 = 1.f - powf(beta1, (float)t);
    const float c2 = 1.f - powf(beta2, (float)t);
    p[k] = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Mean of n values by one workgroup (fixed order) into out[0].
__global__ void __launch_bounds__(256) mlp_mean_kernel(const float *__restrict__ a, int n, float *__restrict__ out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += (double)a[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = (float)(t / (double)n);
}

}  // namespace

int mlp_nparams(int F) { return offsets(F).P; }

size_t mlp_lds_bytes(int F) { return (size_t)offsets(F).P * sizeof(float); }

hipError_t mlp_forward(const MlpBufs &B, const float *X, const int *idx, int n, float *yhat, bool keep,
                       hipStream_t s) {
    const unsigned nb = (unsigned)((n + kMlpThreads - 1) / kMlpThreads);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(nb), dim3(kMlpThreads), mlp_lds_bytes(B.F), s, B.params, B.mu, B.sd,
                       X, idx, n, B.F, keep ? B.xs : nullptr, keep ? B.h1 : nullptr, keep ? B.h2 : nullptr,
                       keep ? B.h3 : nullptr, yhat);
    return hipGetLastError();
}

hipError_t mlp_backward(const MlpBufs &B, const float *y, const int *idx, int n, hipStream_t s) {
    const unsigned nb = (unsigned)((n + kMlpThreads - 1) / kMlpThreads);
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(nb), dim3(kMlpThreads), mlp_lds_bytes(B.F), s, B.params, B.F, y, idx, n,
                       B.yhat, B.h1, B.h2, B.h3, B.g, B.d1, B.d2, B.d3, B.sqerr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int P = mlp_nparams(B.F);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, B.F, n, B.xs, B.h1, B.h2,
                       B.h3, B.g, B.d1, B.d2, B.d3, B.grad);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_mean_kernel, dim3(1), dim3(256), 0, s, B.sqerr, n, B.loss + B.loss_at);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpBufs &B, int t, float lr, hipStream_t s) {
    const int P = mlp_nparams(B.F);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, B.params, B.m, B.v, B.grad,
                       P, t, lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

}  // namespace jk
