// lbm_mlp_device.h -- wavefront-wide evaluation of the eddy-viscosity closure
// network (7 -> 32 -> 32 -> 1, ReLU, softplus) on BF16 matrix cores.
//
// One wavefront evaluates its 64 nodes at once with 16 v_mfma_f32_16x16x32_bf16
// (8 per hidden layer).  Neurons are the M dimension, nodes the N dimension
// (four 16-node tiles per wave).  No lane exchange is needed:
//  - layer 1: for node tile t only lane group t (lanes 16t..16t+15) feeds
//    non-zero operands -- its own node's 7 features and the matching W1 rows
//    -- so the other lane groups' K slots are zero on both sides;
//  - layer 2: the layer-1 accumulator of lane (g, j) holds neurons
//    4g..4g+3 and 16+4g..16+4g+3 of node j of the tile; those eight values
//    are used directly as that lane's K slots, and W2 is stored with its
//    columns permuted the same way (host side, lbm_mlp.hip);
//  - layer 3 (32 -> 1) is a dot product per lane plus two xor-shuffles.
// Only the (row = lane % 16) operand and (col = lane % 16, rows 4*(lane/16)
// + r) accumulator layouts of the 16x16 MFMA matter; the K-slot order of the
// operands cancels because A and B use the same per-lane slots.
//
// Inputs, weights and hidden activations are BF16 (round to nearest even);
// accumulation, biases and normalisation are FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbmd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ float softplus_f(float z) { return z > 20.0f ? z : log1pf(expf(z)); }

// Returns softplus(net(x)) for this lane's node (every lane of the wave must
// call it; lanes whose result is unused may pass any finite features).
__device__ __forceinline__ float mlp_wave_eval(const MlpDev &m, const float feat[7]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, j = lane & 15;

    bf16x8 xo;
#pragma unroll
    for (int k = 0; k < 7; ++k) xo[k] = (__bf16)((feat[k] - m.mean[k]) / m.sd[k]);
    xo[7] = (__bf16)0.0f;
    const bf16x8 zero = {};

    const bf16x8 w1a0 = load_bf16x8(m.w1 + (0 * 16 + j) * 8);
    const bf16x8 w1a1 = load_bf16x8(m.w1 + (1 * 16 + j) * 8);
    const bf16x8 w2a0 = load_bf16x8(m.w2 + ((0 * 4 + g) * 16 + j) * 8);
    const bf16x8 w2a1 = load_bf16x8(m.w2 + ((1 * 4 + g) * 16 + j) * 8);
    const float4 b1a = *reinterpret_cast<const float4 *>(m.b1 + 4 * g);
    const float4 b1b = *reinterpret_cast<const float4 *>(m.b1 + 16 + 4 * g);
    const float4 b2a = *reinterpret_cast<const float4 *>(m.b2 + 4 * g);
    const float4 b2b = *reinterpret_cast<const float4 *>(m.b2 + 16 + 4 * g);
    const float4 w3a = *reinterpret_cast<const float4 *>(m.w3 + 4 * g);
    const float4 w3b = *reinterpret_cast<const float4 *>(m.w3 + 16 + 4 * g);
    const float b3 = m.b3[0];

    float z_own = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool mine = (g == t);
        const bf16x8 B1 = mine ? xo : zero;
        const f32x4 c0 = {0.0f, 0.0f, 0.0f, 0.0f};
        f32x4 h1a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mine ? w1a0 : zero, B1, c0, 0, 0, 0);
        f32x4 h1b = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mine ? w1a1 : zero, B1, c0, 0, 0, 0);
        bf16x8 B2;
        B2[0] = (__bf16)fmaxf(h1a[0] + b1a.x, 0.0f);
        B2[1] = (__bf16)fmaxf(h1a[1] + b1a.y, 0.0f);
        B2[2] = (__bf16)fmaxf(h1a[2] + b1a.z, 0.0f);
        B2[3] = (__bf16)fmaxf(h1a[3] + b1a.w, 0.0f);
        B2[4] = (__bf16)fmaxf(h1b[0] + b1b.x, 0.0f);
        B2[5] = (__bf16)fmaxf(h1b[1] + b1b.y, 0.0f);
        B2[6] = (__bf16)fmaxf(h1b[2] + b1b.z, 0.0f);
        B2[7] = (__bf16)fmaxf(h1b[3] + b1b.w, 0.0f);
        f32x4 h2a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2a0, B2, c0, 0, 0, 0);
        f32x4 h2b = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2a1, B2, c0, 0, 0, 0);
        float part = 0.0f;
        part += w3a.x * (float)(__bf16)fmaxf(h2a[0] + b2a.x, 0.0f);
        part += w3a.y * (float)(__bf16)fmaxf(h2a[1] + b2a.y, 0.0f);
        part += w3a.z * (float)(__bf16)fmaxf(h2a[2] + b2a.z, 0.0f);
        part += w3a.w * (float)(__bf16)fmaxf(h2a[3] + b2a.w, 0.0f);
        part += w3b.x * (float)(__bf16)fmaxf(h2b[0] + b2b.x, 0.0f);
        part += w3b.y * (float)(__bf16)fmaxf(h2b[1] + b2b.y, 0.0f);
        part += w3b.z * (float)(__bf16)fmaxf(h2b[2] + b2b.z, 0.0f);
        part += w3b.w * (float)(__bf16)fmaxf(h2b[3] + b2b.w, 0.0f);
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (mine) z_own = part + b3;
    }
    return softplus_f(z_own);
}

}  // namespace lbmd
