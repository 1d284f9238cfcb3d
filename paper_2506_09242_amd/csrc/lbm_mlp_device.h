// lbm_mlp_device.h -- wavefront-wide evaluation of the eddy-viscosity closure
// network (7 -> 32 -> 32 -> 1, ReLU, softplus) on BF16 matrix cores.
//
// One wavefront evaluates its 64 nodes with six v_mfma_f32_32x32x16_bf16:
// neurons are the M dimension, nodes the N dimension, one half-wave of 32
// nodes per product (lane l's node is node l of the wave, half h = l / 32).
// Only these layouts of the 32x32x16 product are relied on: lane l supplies
// row (l % 32) of A and column (l % 32) of B, eight K slots each (lanes l and
// l + 32 the two halves of K), and its accumulator register r holds output
// row 8 (r / 4) + 4 (l / 32) + r % 4 of column l % 32 (the "accumulator
// order" of lane group l / 32).  The order of the K slots cancels because A
// and B use the same per-lane slots.
//  - layer 1 (K = 7, padded to 8): for half h only the lanes of half h feed
//    non-zero operands -- their own node's features and row l % 32 of W1 --
//    so one product per half (two in all); the accumulator starts from b1;
//  - layer 2 (K = 32): the layer-1 accumulator of lane l holds 16 of the 32
//    neurons of its column's node; registers 0..7 and 8..15 are the K slots
//    of two chained products (accumulator from b2), with W2's columns
//    permuted to that order on the host (two per half);
//  - layer 3 (32 -> 1): eight two-term BF16 dot products per lane over its 16
//    neurons (W3 stored in accumulator order), plus one xor-shuffle with the
//    partner lane l ^ 32, which holds the other 16.
// ReLU acts on the BF16-rounded activations (rounding keeps the sign, so this
// equals rounding the rectified value): a packed 16-bit signed max with 0.
// Inputs, weights and hidden activations are BF16 (round to nearest even);
// accumulation, biases and normalisation are FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbmd {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// softplus(z) = ln(1 + e^z) from the hardware base-2 exponential and
// logarithm (v_exp_f32, v_log_f32): ln 2 * log2(1 + t), t = 2^(z log2 e);
// for z < -5, where 1 + t loses t's low bits, t (1 - t/2) instead (relative
// error below t^2/3 < 2e-5); z itself above 15 (error below e^-15).
__device__ __forceinline__ float softplus_f(float z) {
    const float t = __builtin_amdgcn_exp2f(z * 1.44269504088896341f);
    const float mid = 0.693147180559945309f * __builtin_amdgcn_logf(1.0f + t);
    return z > 15.0f ? z : (z < -5.0f ? t * (1.0f - 0.5f * t) : mid);
}

// max(RNE_bf16(a), 0), max(RNE_bf16(b), 0): a negative BF16 pattern is a
// negative 16-bit integer, so a signed max with 0 is the ReLU.
__device__ __forceinline__ bf16x2 relu_bf16x2(float a, float b) {
    const f32x2 f = {a, b};
    const bf16x2 v = __builtin_convertvector(f, bf16x2);  // one paired RNE conversion
    const s16x2 z = {0, 0};
    return __builtin_bit_cast(bf16x2, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), z));
}

// Eight accumulator registers starting at r0 -> eight BF16 K slots.
template <int R0>
__device__ __forceinline__ bf16x8 relu_slots(const f32x16 &acc) {
    bf16x8 k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x2 v = relu_bf16x2(acc[R0 + 2 * q], acc[R0 + 2 * q + 1]);
        k[2 * q] = v[0];
        k[2 * q + 1] = v[1];
    }
    return k;
}

// 16 floats of this lane group's accumulator-order vector (biases).
__device__ __forceinline__ f32x16 load_acc_order(const float *p) {
    f32x16 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 t = reinterpret_cast<const float4 *>(p)[q];
        v[4 * q] = t.x;
        v[4 * q + 1] = t.y;
        v[4 * q + 2] = t.z;
        v[4 * q + 3] = t.w;
    }
    return v;
}

// Returns softplus(net(x)) for this lane's node (every lane of the wave must
// call it; lanes whose result is unused may pass any finite features).
__device__ __forceinline__ float mlp_wave_eval(const MlpDev &m, const float feat[7]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5, j = lane & 31;

    bf16x8 xo;
#pragma unroll
    for (int k = 0; k < 7; ++k) xo[k] = (__bf16)((feat[k] - m.mean[k]) * m.inv_sd[k]);
    xo[7] = (__bf16)0.0f;
    const bf16x8 zero = {};
    const bf16x8 w1 = load_bf16x8(m.w1 + j * 8);
    const f32x16 c1 = load_acc_order(m.b1 + 16 * g);
    const f32x16 c2 = load_acc_order(m.b2 + 16 * g);
    const uint4 w3a = reinterpret_cast<const uint4 *>(m.w3 + 16 * g)[0];
    const uint4 w3b = reinterpret_cast<const uint4 *>(m.w3 + 16 * g)[1];
    const bf16x2 w3[8] = {__builtin_bit_cast(bf16x2, w3a.x), __builtin_bit_cast(bf16x2, w3a.y),
                          __builtin_bit_cast(bf16x2, w3a.z), __builtin_bit_cast(bf16x2, w3a.w),
                          __builtin_bit_cast(bf16x2, w3b.x), __builtin_bit_cast(bf16x2, w3b.y),
                          __builtin_bit_cast(bf16x2, w3b.z), __builtin_bit_cast(bf16x2, w3b.w)};

    float z_own = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const bool mine = (g == h);
        const f32x16 h1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mine ? w1 : zero, mine ? xo : zero, c1, 0, 0, 0);
        f32x16 h2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(m.w2 + ((0 * 2 + g) * 32 + j) * 8),
                                                            relu_slots<0>(h1), c2, 0, 0, 0);
        h2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(m.w2 + ((1 * 2 + g) * 32 + j) * 8),
                                                     relu_slots<8>(h1), h2, 0, 0, 0);
        float part = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            part = __builtin_amdgcn_fdot2_f32_bf16(relu_bf16x2(h2[2 * q], h2[2 * q + 1]), w3[q], part, false);
        part += __shfl_xor(part, 32, 64);
        if (mine) z_own = part + m.b3[0];
    }
    return softplus_f(z_own);
}

}  // namespace lbmd
