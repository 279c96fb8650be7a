// Wave-level evaluation of the path-length MLP on the matrix cores.  The
// register layout is described in mlp.h.  All 64 lanes of the wave must
// execute these functions together (MFMA is a whole-wave operation).
#pragma once
#include "mlp.h"

namespace p2r {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma32(const bf16x8& a, const bf16x8& b, const floatx16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p) {
    bf16x8 v;
    __builtin_memcpy(&v, p, sizeof v);
    return v;
}

// row of element j of a 32x32 output block in lane half hi
__device__ __forceinline__ int blk_row(int j, int hi) { return 8 * (j >> 2) + 4 * hi + (j & 3); }

__device__ __forceinline__ floatx16 bias_init(const float* b, int base, int hi) {
    floatx16 c;
#pragma unroll
    for (int j = 0; j < 16; ++j) c[j] = b[base + blk_row(j, hi)];
    return c;
}

// max(x, 0) as one integer max on the bit pattern: a float with its sign bit
// set is a negative integer, so it becomes +0 and every other value passes
// unchanged.  (fmaxf costs two instructions here: the compiler first
// quiets a possible signalling NaN, which the pre-activations, sums of
// finite products, never are.)
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ bf16x8 relu_bf16(const floatx16& a, int from) {
    bf16x8 v;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (__bf16)relu(a[from + k]);
    return v;
}

// z1[mb][nb], z2[mb][nb] pre-activations; returns y for this lane's sample.
struct MlpActs {
    floatx16 z1[2][2];
    floatx16 z2[2][2];
};

__device__ __forceinline__ float mlp_eval(const MlpWeights& W, const float feat[MLP_IN], MlpActs* keep) {
    const int l = __lane_id();
    const int hi = l >> 5;
    const int r32 = l & 31;
    bf16x8 xb;
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) xb[k] = (__bf16)(isfinite(feat[k]) ? feat[k] : 0.0f);
    xb[7] = (__bf16)0.0f;
    const bf16x8 zero = {};
    floatx16 z1[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const bf16x8 w = load_bf16x8(&W.w1[mb * 32 + r32][0]);
        const floatx16 c0 = bias_init(W.b1, mb * 32, hi);
        z1[mb][0] = mfma32(hi ? zero : w, xb, c0);
        z1[mb][1] = mfma32(hi ? w : zero, xb, c0);
    }
    floatx16 z2[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const floatx16 c0 = bias_init(W.b2, mb * 32, hi);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = c0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bf16x8 a = load_bf16x8(&W.w2[mb][c][r32][8 * hi]);
                const bf16x8 b = relu_bf16(z1[c >> 1][nb], 8 * (c & 1));
                acc = mfma32(a, b, acc);
            }
            z2[mb][nb] = acc;
        }
    }
    float part[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        float s = 0.0f;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int j = 0; j < 16; ++j) s = fmaf(W.w3[mb * 32 + blk_row(j, hi)], relu(z2[mb][nb][j]), s);
        part[nb] = s + __shfl_xor(s, 32);
    }
    if (keep) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) { keep->z1[a][b] = z1[a][b]; keep->z2[a][b] = z2[a][b]; }
    }
    return (hi ? part[1] : part[0]) + W.b3;
}

// Inference only, with few live registers (fused into the fit kernel):
// layer-1 activations are kept as BF16 B operands, and each layer-2 block is
// folded into the output as soon as it is complete.
__device__ __forceinline__ float mlp_infer(const MlpWeights& W, const float feat[MLP_IN]) {
    const int l = __lane_id();
    const int hi = l >> 5;
    const int r32 = l & 31;
    bf16x8 xb;
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) xb[k] = (__bf16)feat[k];
    xb[7] = (__bf16)0.0f;
    const bf16x8 zero = {};
    bf16x8 h1[2][2][2];   // [row block][column block][half of the block]
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const bf16x8 w = load_bf16x8(&W.w1[mb * 32 + r32][0]);
        const floatx16 c0 = bias_init(W.b1, mb * 32, hi);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const floatx16 z = mfma32(nb == 0 ? (hi ? zero : w) : (hi ? w : zero), xb, c0);
            h1[mb][nb][0] = relu_bf16(z, 0);
            h1[mb][nb][1] = relu_bf16(z, 8);
        }
    }
    float part[2] = {0.0f, 0.0f};
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const floatx16 c0 = bias_init(W.b2, mb * 32, hi);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = c0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc = mfma32(load_bf16x8(&W.w2[mb][c][r32][8 * hi]), h1[c >> 1][nb][c & 1], acc);
#pragma unroll
            for (int j = 0; j < 16; ++j) part[nb] = fmaf(W.w3[mb * 32 + blk_row(j, hi)], relu(acc[j]), part[nb]);
        }
    }
    const float s0 = part[0] + __shfl_xor(part[0], 32);
    const float s1 = part[1] + __shfl_xor(part[1], 32);
    return (hi ? s1 : s0) + W.b3;
}

// The 7 features of a (state, target cylinder) pair (the network's input)
// and the straight-line path s_line = (R^2 - r0^2) / (b + sqrt(b^2 + R^2 - r0^2)):
//   [r0/R, b/R, a/R, omega R, s_line/R, omega s_line, omega a],
// b = x cos(phi) + y sin(phi), a = y cos(phi) - x sin(phi).  Returns false
// (features zeroed) when the line does not reach R outward.
__device__ __forceinline__ bool mlp_features_of(float x, float y, float cphi, float sphi, float w, float R,
                                                float feat[MLP_IN], float& s_line) {
    const float b = x * cphi + y * sphi;
    const float a = y * cphi - x * sphi;
    const float r0sq = fmaf(x, x, y * y);
    const float dr2 = R * R - r0sq;
    const float den = b + sqrtf(fmaxf(fmaf(b, b, dr2), 0.0f));
    const bool ok = dr2 > 0.0f && den > 0.0f;
    s_line = ok ? dr2 / den : 0.0f;
    const float iR = 1.0f / R;
    // a non-finite feature would spoil the whole 32-sample column block of the
    // matrix product (0 * inf), so features are clamped and zeroed when invalid
    feat[0] = sqrtf(r0sq) * iR;
    feat[1] = b * iR;
    feat[2] = a * iR;
    feat[3] = w * R;
    feat[4] = s_line * iR;
    feat[5] = w * s_line;
    feat[6] = w * a;
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) feat[k] = ok && isfinite(feat[k]) ? fminf(fmaxf(feat[k], -1e4f), 1e4f) : 0.0f;
    return ok;
}

}  // namespace p2r
