// gwfa_mlp.hip -- training and batch inference of the diagonal keep/drop
// network used by the learned pruning mode (8 -> 64 ReLU -> 64 ReLU -> 1).
//
// The forward pass is the inference arithmetic of gwfa_mlp_dev.h: inputs
// x = bf16(feature * scale), bfloat16 weights, activations rounded to
// bfloat16 after each ReLU, float32 sums in the same order, so a trained
// network scores a diagonal in training exactly as the alignment kernel does.
// Loss: binary cross-entropy on the logit, positives weighted by pos_weight,
// averaged over the samples of the call.  The backward pass treats the
// bfloat16 roundings as the identity.  Adam keeps float32 master weights and
// moments and writes the bfloat16 copy the kernels read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gwfa_internal.h"
#include "gwfa_mlp_dev.h"

namespace gwfa_train {

using namespace gwfa_nn;

// per-sample activations kept between the two passes:
// x[8] | h1[64] | h2[64] | g2[64] = dL/da2 | g1[64] = dL/da1 | dz = dL/dz
constexpr int C_X = 0, C_H1 = 8, C_H2 = 72, C_G2 = 136, C_G1 = 200, C_DZ = 264, SS = 265;
constexpr int SPB = 256;   // samples per block of the weight-gradient kernel

__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoid(float z) {
    const float e = expf(-fabsf(z));
    return z >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
}

__global__ void k_zero(float* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Forward and per-sample backward, one thread per sample.
__global__ __launch_bounds__(256) void k_act(const float* __restrict__ feat, int64_t stride, Scale8 scale,
                                             const uint8_t* __restrict__ label, int64_t n, float pos_weight,
                                             float inv_n, const uint16_t* __restrict__ w, float* __restrict__ scr,
                                             float* __restrict__ loss) {
    __shared__ float sw[MLP_N];
    __shared__ float part[4];
    for (int i = threadIdx.x; i < MLP_N; i += blockDim.x) sw[i] = bf2f(w[i]);
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float my_loss = 0.0f;
    if (b < n) {
        float* S = scr + b * SS;
        const float* f = feat + b * stride;
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            x[i] = round_bf16(f[i] * scale.s[i]);
            S[C_X + i] = x[i];
        }
        float h1[64];
        unsigned long long m1 = 0, m2 = 0;   // ReLU masks
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            float a = sw[MW_B1 + j];
#pragma unroll
            for (int i = 0; i < 8; ++i) a = fmaf(sw[j * 8 + i], x[i], a);
            if (a > 0.0f) m1 |= 1ull << j;
            h1[j] = round_bf16(fmaxf(a, 0.0f));
            S[C_H1 + j] = h1[j];
        }
        float z = sw[MW_B3];
        for (int j = 0; j < 64; ++j) {
            float a = sw[MW_B2 + j];
#pragma unroll
            for (int k = 0; k < 64; ++k) a = fmaf(sw[MW_W2 + j * 64 + k], h1[k], a);
            if (a > 0.0f) m2 |= 1ull << j;
            const float h2 = round_bf16(fmaxf(a, 0.0f));
            S[C_H2 + j] = h2;
            z = fmaf(sw[MW_W3 + j], h2, z);
        }
        const bool pos = label[b] != 0;
        my_loss = pos ? pos_weight * softplus(-z) : softplus(z);
        const float sz = sigmoid(z);
        const float dz = (pos ? pos_weight * (sz - 1.0f) : sz) * inv_n;
        S[C_DZ] = dz;
        float g2[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            g2[j] = ((m2 >> j) & 1) ? dz * sw[MW_W3 + j] : 0.0f;
            S[C_G2 + j] = g2[j];
        }
        for (int k = 0; k < 64; ++k) {
            float a = 0.0f;
#pragma unroll
            for (int j = 0; j < 64; ++j) a = fmaf(sw[MW_W2 + j * 64 + k], g2[j], a);
            S[C_G1 + k] = ((m1 >> k) & 1) ? a : 0.0f;
        }
    }
    // block sum of the loss: wave sums, then one atomic per block
    float v = my_loss;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) * inv_n);
}

// Weight gradients: thread = parameter, block row = SPB samples.
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ scr, int64_t n, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.y * SPB;
    if (p >= MLP_N || b0 >= n) return;
    int ca, cb;   // columns multiplied; cb < 0: column ca alone
    if (p < MW_B1) { ca = C_G1 + p / 8; cb = C_X + p % 8; }                         // W1[j][i]
    else if (p < MW_W2) { ca = C_G1 + (p - MW_B1); cb = -1; }                       // b1[j]
    else if (p < MW_B2) { ca = C_G2 + (p - MW_W2) / 64; cb = C_H1 + (p - MW_W2) % 64; }   // W2[j][k]
    else if (p < MW_W3) { ca = C_G2 + (p - MW_B2); cb = -1; }                       // b2[j]
    else if (p < MW_B3) { ca = C_DZ; cb = C_H2 + (p - MW_W3); }                     // W3[j]
    else { ca = C_DZ; cb = -1; }                                                    // b3
    const int64_t b1 = min(n, b0 + SPB);
    float acc = 0.0f;
    for (int64_t b = b0; b < b1; ++b) {
        const float* S = scr + b * SS;
        acc = fmaf(S[ca], cb >= 0 ? S[cb] : 1.0f, acc);
    }
    atomicAdd(&grad[p], acc);
}

__global__ void k_adam(float* __restrict__ master, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ grad, uint16_t* __restrict__ wb, float lr, float beta1, float beta2,
                       float eps, float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_N) return;
    const float g = grad[p];
    const float a = beta1 * m1[p] + (1.0f - beta1) * g;
    const float b = beta2 * m2[p] + (1.0f - beta2) * g * g;
    m1[p] = a;
    m2[p] = b;
    const float upd = (a / bc1) / (sqrtf(b / bc2) + eps);
    const float w = master[p] - lr * upd;
    master[p] = w;
    wb[p] = f2bf(w);
}

__global__ void k_cast(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

// Logits of n samples with the alignment kernel's inference routine.
__global__ __launch_bounds__(256) void k_logits(const float* __restrict__ feat, int64_t stride, Scale8 scale,
                                                int64_t n, const uint16_t* __restrict__ w, float* __restrict__ out) {
    __shared__ __align__(16) uint16_t sw[MLP_N + 7];
    for (int i = threadIdx.x; i < MLP_N; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    // every lane of the wave takes part in the matrix products
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (b < n) {
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = feat[b * stride + i];
    }
    const float z = mlp_logit_wave(f, scale.s, sw);
    if (b < n) out[b] = z;
}

}  // namespace gwfa_train

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
int64_t gwfa_mlp_scratch_floats(int64_t samples) { return samples * gwfa_train::SS; }

hipError_t gwfa_launch_mlp_grad(const float* feat, int64_t stride, const Scale8& scale, const uint8_t* label,
                                int64_t n, float pos_weight, const uint16_t* w, float* scr, int64_t scr_samples,
                                float* grad, float* loss, hipStream_t st) {
    using namespace gwfa_train;
    (void)hipGetLastError();   // report only this call's launch status
    hipLaunchKernelGGL(k_zero, dim3((MLP_N + 255) / 256), dim3(256), 0, st, grad, MLP_N);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, loss, 1);
    if (n <= 0) return hipGetLastError();
    const float inv_n = 1.0f / (float)n;
    for (int64_t c0 = 0; c0 < n; c0 += scr_samples) {
        const int64_t m = std::min<int64_t>(scr_samples, n - c0);
        hipLaunchKernelGGL(k_act, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, feat + c0 * stride, stride,
                           scale, label + c0, m, pos_weight, inv_n, w, scr, loss);
        hipLaunchKernelGGL(k_wgrad, dim3((MLP_N + 255) / 256, (unsigned)((m + SPB - 1) / SPB)), dim3(256), 0, st, scr,
                           m, grad);
    }
    return hipGetLastError();
}

hipError_t gwfa_launch_mlp_adam(float* master, float* m1, float* m2, const float* grad, uint16_t* wb, float lr,
                                float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t st) {
    using namespace gwfa_train;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_adam, dim3((MLP_N + 255) / 256), dim3(256), 0, st, master, m1, m2, grad, wb, lr, beta1,
                       beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t gwfa_launch_mlp_cast(const float* src, uint16_t* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_train::k_cast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t gwfa_launch_mlp_logits(const float* feat, int64_t stride, const Scale8& scale, int64_t n,
                                  const uint16_t* w, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_train::k_logits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, feat, stride, scale,
                       n, w, out);
    return hipGetLastError();
}
