// Step-predictor MLP 8 -> 32 -> 32 -> 1 (ReLU), output
// omega = 1 + (omega_max - 1) * sigmoid(z).  Not part of the paper: it
// proposes over-relaxed sphere-tracing steps that the tracer accepts only when
// the unbounding spheres of both ends overlap (the over-relaxation test the
// paper cites, Keinert et al. 2014), so the plain step stays the fallback.
//
// Parameters: 1377 floats, layout W1[32][8], b1[32], W2[32][32], b2[32],
// w3[32], b3.  Arithmetic: binary16 inputs and weights, FP32 accumulation,
// hidden activations rounded to binary16 after the ReLU.
//
// Inference runs on the matrix cores for the 64 rays of a wave, as two blocks
// of 32 rays, in transposed form: H1^T = W1 . X^T and H2^T = W2 . H1^T with
// v_mfma_f32_32x32x8_f16.  In that form the accumulator registers of layer 1
// (lane l: ray l % 32, hidden rows 8q + 4(l/32) + r, q, r in 0..3) are exactly
// the B operand of layer 2's K-chunk q, so no shuffles are needed between the
// layers.  Layer 3 (32 -> 1) is a VALU dot product completed across the two
// half-waves.
#pragma once

#include "st_common.h"

namespace st {

constexpr int kMlpParams = 1377;
constexpr int kMlpW1 = 0, kMlpB1 = 256, kMlpW2 = 288, kMlpB2 = 1312, kMlpW3 = 1344, kMlpB3 = 1376;
constexpr float kOmegaMax = 4.0f;
constexpr float kFeatClamp = 3.0f;   // standardised features are clamped to [-3, 3]
// the tracer runs the model once every kMlpEvery stepping iterations of a
// wave (the inference costs about as much as a small view's evaluation)
constexpr int kMlpEvery = 4;

// Per-lane operand table, one column per lane (entry k of lane l at k*64+l):
//  [0,1]   W1 A operand: halves W1[h][4g..4g+3]          (h = l % 32, g = l / 32)
//  [2..9]  W2 A operands, chunk c: halves W2[h][8c+4g..+3]
//  [10..25] b1 at the accumulator rows 8(a/4)+4g+a%4, a = 0..15
//  [26..41] b2 at the same rows
//  [42..57] w3 at the same rows
//  [58]    b3
// followed by 16 floats: feature means[8], inverse standard deviations[8].
constexpr int kMlpTabRows = 59;
constexpr int kMlpTabWords = kMlpTabRows * 64 + 16;

typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int mlp_row(int a, int g) { return 8 * (a >> 2) + 4 * g + (a & 3); }

__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
    _Float16 x = (_Float16)a, y = (_Float16)b;
    return uint32_t(__builtin_bit_cast(uint16_t, x)) | (uint32_t(__builtin_bit_cast(uint16_t, y)) << 16);
}
__device__ __forceinline__ h4_t h4_from(uint32_t lo, uint32_t hi) {
    typedef uint32_t u2_t __attribute__((ext_vector_type(2)));
    u2_t u = {lo, hi};
    return __builtin_bit_cast(h4_t, u);
}
__device__ __forceinline__ float round_half(float x) { return float((_Float16)x); }

// omega for the ray of this lane.  tab: the operand table (LDS or global; 32-bit
// words, floats stored as their bits), x: the 8 raw features of this lane's
// ray.  Must be called with all 64 lanes of the wave active (matrix
// instructions and cross-lane shuffles).
__device__ __forceinline__ float tabf(const uint32_t* tab, int k) { return __uint_as_float(tab[k]); }

// standardised feature, clamped so that an input far outside the training
// range stays finite in binary16
__device__ __forceinline__ float mlp_feature(float x, float mean, float inv_std) {
    return fminf(fmaxf((x - mean) * inv_std, -kFeatClamp), kFeatClamp);
}

__device__ __forceinline__ float mlp_omega(const uint32_t* tab, const float x[8]) {
    const int l = int(threadIdx.x & 63u), g = l >> 5;
    const uint32_t* nrm = tab + kMlpTabRows * 64;
    float xn[8];
#pragma unroll
    for (int i = 0; i < 8; i++) xn[i] = mlp_feature(x[i], tabf(nrm, i), tabf(nrm, 8 + i));
    uint32_t lo0 = pack_h2(xn[0], xn[1]), lo1 = pack_h2(xn[2], xn[3]);
    uint32_t hi0 = pack_h2(xn[4], xn[5]), hi1 = pack_h2(xn[6], xn[7]);
    uint32_t slo0 = __shfl_xor(lo0, 32), slo1 = __shfl_xor(lo1, 32);
    uint32_t shi0 = __shfl_xor(hi0, 32), shi1 = __shfl_xor(hi1, 32);
    // B operands: block 0 = rays 0..31, block 1 = rays 32..63; lane l holds
    // features 4g..4g+3 of ray 32b + l%32
    const h4_t B0 = g == 0 ? h4_from(lo0, lo1) : h4_from(shi0, shi1);
    const h4_t B1 = g == 0 ? h4_from(slo0, slo1) : h4_from(hi0, hi1);
    float z = 0.f;
    // the two blocks one after the other: 32 accumulators live, not 64
#pragma unroll 1
    for (int blk = 0; blk < 2; blk++) {
        const h4_t B = blk == 0 ? B0 : B1;
        f16_t c;
#pragma unroll
        for (int a = 0; a < 16; a++) c[a] = tabf(tab, (10 + a) * 64 + l);
        const f16_t d = __builtin_amdgcn_mfma_f32_32x32x8f16(h4_from(tab[l], tab[64 + l]), B, c, 0, 0, 0);
        f16_t e;
#pragma unroll
        for (int a = 0; a < 16; a++) e[a] = tabf(tab, (26 + a) * 64 + l);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const h4_t A2 = h4_from(tab[(2 + 2 * q) * 64 + l], tab[(3 + 2 * q) * 64 + l]);
            const h4_t b = h4_from(pack_h2(fmaxf(d[4 * q], 0.f), fmaxf(d[4 * q + 1], 0.f)),
                                   pack_h2(fmaxf(d[4 * q + 2], 0.f), fmaxf(d[4 * q + 3], 0.f)));
            e = __builtin_amdgcn_mfma_f32_32x32x8f16(A2, b, e, 0, 0, 0);
        }
        float p = 0.f;
#pragma unroll
        for (int a = 0; a < 16; a++) p = fmaf(tabf(tab, (42 + a) * 64 + l), round_half(fmaxf(e[a], 0.f)), p);
        p += __shfl_xor(p, 32);
        if (g == blk) z = p;
    }
    z += tabf(tab, 58 * 64 + l);
    return 1.0f + (kOmegaMax - 1.0f) / (1.0f + __expf(-z));
}

}  // namespace st
