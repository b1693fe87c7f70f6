// gwfa_mlp_dev.h -- device arithmetic of the diagonal keep/drop network,
// shared by the fused inference in the alignment kernel and the training
// kernels.  Network: 8 -> 64 ReLU -> 64 ReLU -> 1 logit; weights and
// activations are bfloat16 values (rounded to nearest, ties to even), sums
// are float32 fused multiply-adds in a fixed order.
// Weight layout: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwfa_nn {

constexpr int MLP_N = 4801;
constexpr int MW_B1 = 512, MW_W2 = 576, MW_B2 = 4672, MW_W3 = 4736, MW_B3 = 4800;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// round to the nearest bfloat16 (ties to even), kept in a float
__device__ __forceinline__ float round_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ uint16_t f2bf(float x) {
    return (uint16_t)(__float_as_uint(round_bf16(x)) >> 16);
}

// logit of one entry: x = bf16(f * scale); the order of every sum is the
// order of the loops below
__device__ __forceinline__ float mlp_logit(const float* f, const float* scale, const uint16_t* w) {
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = round_bf16(f[i] * scale[i]);
    // first-layer activations as packed bfloat16 pairs (32 registers)
    uint32_t h1[32];
#pragma unroll
    for (int j2 = 0; j2 < 32; ++j2) {
        float a0 = bf2f(w[MW_B1 + 2 * j2]), a1 = bf2f(w[MW_B1 + 2 * j2 + 1]);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a0 = fmaf(bf2f(w[(2 * j2) * 8 + i]), x[i], a0);
            a1 = fmaf(bf2f(w[(2 * j2 + 1) * 8 + i]), x[i], a1);
        }
        h1[j2] = (__float_as_uint(round_bf16(fmaxf(a0, 0.0f))) >> 16) |
                 (__float_as_uint(round_bf16(fmaxf(a1, 0.0f))) & 0xffff0000u);
    }
    float z = bf2f(w[MW_B3]);
#pragma unroll 1
    for (int j = 0; j < 64; ++j) {
        float acc = bf2f(w[MW_B2 + j]);
        const uint32_t* row = reinterpret_cast<const uint32_t*>(w + MW_W2 + j * 64);
#pragma unroll
        for (int m = 0; m < 32; ++m) {
            const uint32_t wp = row[m];
            acc = fmaf(__uint_as_float(wp << 16), __uint_as_float(h1[m] << 16), acc);
            acc = fmaf(__uint_as_float(wp & 0xffff0000u), __uint_as_float(h1[m] & 0xffff0000u), acc);
        }
        z = fmaf(bf2f(w[MW_W3 + j]), round_bf16(fmaxf(acc, 0.0f)), z);
    }
    return z;
}

// The same as a call of its own: its registers then do not add to those of
// the alignment loop around it (inlined into a 64-lane workgroup's loop the
// compiler spills hundreds of registers); where inlining fits, the call's
// overhead is not worth paying.
__device__ __attribute__((noinline)) float mlp_logit_call(const float* f, const float* scale, const uint16_t* w) {
    return mlp_logit(f, scale, w);
}

}  // namespace gwfa_nn
