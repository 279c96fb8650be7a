// Path-length MLP: 7 -> 64 -> 64 -> 1, ReLU, BF16 operands on the matrix
// cores (v_mfma_f32_32x32x16_bf16) with FP32 accumulation and FP32 biases.
//
// Register layout used by every MLP kernel: one wave holds 64 samples, one
// per lane.  A 32x32 MFMA output block gives lane l the column (sample)
// l % 32 and the 16 rows 8 (j / 4) + 4 (l / 32) + j % 4, j = 0..15.
// Layer 1 computes h1^T = W1 x^T with the weights as the A operand: for the
// column block of samples 0..31 the lanes 0..31 supply their own features as
// K = 0..7 and lanes 32..63 supply zeros; for samples 32..63 the roles swap,
// so every lane only ever supplies its own sample (two weight copies, one
// with the weights in K 0..7 and one in K 8..15).  Layer 2 contracts over the
// hidden units in the order they already sit in the registers: K-chunk c of
// column block nb is lane l's rows of layer-1 block (c / 2, nb) with
// j in {2 (c % 2), 2 (c % 2) + 1}, and W2's columns are permuted to match
// when the BF16 copy is made, so no activation ever moves between lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2r {

constexpr int MLP_IN = 7;
constexpr int MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 4737
// offsets of the flat parameter vector
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_H;

constexpr float MLP_TARGET_SCALE = 100.0f;   // the network predicts asinh(100 (s / s_line - 1))
constexpr float MLP_ACCEPT_CM = 1e-3f;        // proposals with |r(s0) - R| above this are rejected
constexpr float KAPPA_MLP = 2.99792458e-3f;  // GeV / (T cm)

// Hidden unit behind K index k (0..15) of K-chunk c (0..3) in the layer-2
// register order (see the layout note above).
__host__ __device__ constexpr int mlp_kperm(int c, int k) {
    return (c >> 1) * 32 + 16 * (c & 1) + 8 * ((k & 7) >> 2) + 4 * (k >> 3) + (k & 3);
}

// Device-side weights as the kernels read them (one contiguous block).
struct MlpWeights {
    uint16_t w1[MLP_H][8];         // BF16 A operand of layer 1: [hidden][k], k = 0..6 weights, 7 = 0
    uint16_t w2[2][4][32][16];     // BF16 A operands of layer 2: [row block][K chunk][row][k], columns permuted
    uint16_t w2t[2][4][32][16];    // BF16 A operands of W2^T (backward), rows of W2 permuted alike
    float b1[MLP_H];
    float b2[MLP_H];
    float w3[MLP_H];
    float b3;
    float pad[3];
};

struct MlpDev {
    float* master;   // [MLP_NPARAM] FP32 weights
    float* m;        // Adam first moments
    float* v;        // Adam second moments
    float* grad;     // [MLP_NPARAM] gradient accumulator
    float* loss;     // [1]
    MlpWeights* w;   // BF16 / FP32 copies the kernels use
    float* part;     // [part_blocks][MLP_NPARAM + 1] per-workgroup partial gradients
    int32_t part_blocks;
    int32_t step;
};

int mlp_grad_blocks(int32_t B);

hipError_t mlp_recast(const MlpDev& d, hipStream_t s);
hipError_t mlp_forward(const MlpDev& d, const float* x, float* y, int32_t B, hipStream_t s);
hipError_t mlp_grads(const MlpDev& d, const float* x, const float* t, int32_t B, hipStream_t s);
hipError_t mlp_adam(const MlpDev& d, float lr, int32_t step, hipStream_t s);
hipError_t mlp_features(int32_t n, const float* par, const float* q, const float* R, const float* s_label,
                        float bz, float* x, float* t, float* s_line, hipStream_t s);

}  // namespace p2r
