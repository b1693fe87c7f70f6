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

// ---------------------------------------------------------------------------
// The same network for the 64 entries of a wave at once, on the matrix
// cores.  Every lane of the wave calls it together (uniform control flow,
// all 64 lanes active) with its own entry's features and gets its entry's
// logit.  Entries are taken 16 at a time (four tiles t); all products are
// v_mfma_f32_16x16x32_bf16 (bfloat16 operands, float32 sums):
//   layer 1, transposed: for each block c of 16 units, h1^T = W1 X^T with
//     the 8 inputs in the first 8 of the 32 product positions (the rest
//     zero), so lane (g = l/16, m = l%16) ends with units 16c + 4g + i of
//     entry 16t + m;
//   layer 2: for each block of 16 outputs, two products over the 64 units;
//     the units a lane already holds fill its product positions (units
//     32ks + 4g + i and 32ks + 16 + 4g + i for position block ks), and the
//     weights are gathered in the same order, so no data moves between
//     lanes;
//   layer 3: per entry, a sum over the 16 lanes of a row group.
// Weights, biases and roundings are those of mlp_logit; only the order of
// the float32 sums differs.  w: the 4801 weights, 16-byte aligned.
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ __bf16 bf_of(float x) {   // x already a bfloat16 value
    return __builtin_bit_cast(__bf16, (uint16_t)(__float_as_uint(x) >> 16));
}
__device__ __forceinline__ __bf16 bf_bits(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

__device__ __forceinline__ float mlp_logit_wave(const float* f, const float* scale, const uint16_t* w) {
    const int lane = __lane_id();
    const int col = lane & 15;
    const int grp = lane >> 4;
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = round_bf16(f[i] * scale[i]);
    const __bf16 zero = bf_bits(0);
    const float b3 = bf2f(w[MW_B3]);
    float z_out = 0.0f;
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        // X^T of the tile: lane (0, m) holds the inputs of entry 16t + m
        bf16x8 xb;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float xi = __shfl(x[i], 16 * t + col, 64);
            xb[i] = grp == 0 ? bf_of(xi) : zero;
        }
        float h[16];   // h[4c + i]: unit 16c + 4*grp + i of entry 16t + col
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bf16x8 wa;   // W1 row 16c + col in lanes of group 0
#pragma unroll
            for (int i = 0; i < 8; ++i) wa[i] = grp == 0 ? bf_bits(w[(16 * c + col) * 8 + i]) : zero;
            f32x4 d;
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = bf2f(w[MW_B1 + 16 * c + 4 * grp + i]);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, xb, d, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) h[4 * c + i] = round_bf16(fmaxf(d[i], 0.0f));
        }
        f32x4 acc[4];
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
            const float b = bf2f(w[MW_B2 + 16 * c2 + col]);
            acc[c2] = f32x4{b, b, b, b};
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = bf_of(h[4 * (2 * ks) + i]);
                a[4 + i] = bf_of(h[4 * (2 * ks + 1) + i]);
            }
#pragma unroll
            for (int c2 = 0; c2 < 4; ++c2) {
                const uint16_t* row = w + MW_W2 + (16 * c2 + col) * 64 + 32 * ks + 4 * grp;
                bf16x8 b;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    b[i] = bf_bits(row[i]);
                    b[4 + i] = bf_bits(row[16 + i]);
                }
                acc[c2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c2], 0, 0, 0);
            }
        }
        // third layer: rows 4*grp + i of the tile, summed over the group's 16 lanes
        float p[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float q = 0.0f;
#pragma unroll
            for (int c2 = 0; c2 < 4; ++c2)
                q = fmaf(bf2f(w[MW_W3 + 16 * c2 + col]), round_bf16(fmaxf(acc[c2][i], 0.0f)), q);
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) q += __shfl_xor(q, o, 64);
            p[i] = q;
        }
        // entry 16t + m (m = lane & 15) is row m: group m >> 2, register m & 3
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = __shfl(p[i], 16 * (col >> 2), 64);
        const int ii = lane & 3;
        const float mine = ii == 0 ? v[0] : (ii == 1 ? v[1] : (ii == 2 ? v[2] : v[3]));
        if (grp == t) z_out = b3 + mine;
    }
    return z_out;
}

// The same as a call of its own: its registers then do not add to those of
// the alignment loop around it (inlined there, the compiler spills the
// loop's registers around the matrix products).
__device__ __attribute__((noinline)) float mlp_logit_wave_call(const float* f, const float* scale, const uint16_t* w) {
    return mlp_logit_wave(f, scale, w);
}

}  // namespace gwfa_nn
