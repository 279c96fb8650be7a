// Training and inference kernels of the path-length MLP (layout in mlp.h).
//   forward:  z1 = W1 x + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2),
//             y = w3 . h2 + b3; BF16 operands (x, W1, h1, W2) on the matrix
//             cores, FP32 accumulation, FP32 biases and last layer.
//   backward: dy = 2 (y - t) / B (mean squared error), dz2 = dy w3 * [z2 > 0],
//             dh1 = W2^T dz2 on the matrix cores (BF16 W2, dz2), dz1 = dh1 * [z1 > 0];
//             weight gradients dW2 = dz2 h1^T and dW1 = dz1 x^T on the matrix
//             cores (BF16 dz2, h1, dz1, x; FP32 accumulation), the bias and
//             last-layer sums in FP32 on the vector units.
//   Adam on the FP32 master weights, then a fresh BF16 copy.
#include "mlp.h"
#include "mlp_dev.h"

namespace p2r {

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    __bf16 b = (__bf16)f;
    uint16_t u;
    __builtin_memcpy(&u, &b, 2);
    return u;
}

__global__ void mlp_recast_kernel(const float* __restrict__ P, MlpWeights* __restrict__ W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_H * 8) {
        const int h = i >> 3, k = i & 7;
        W->w1[h][k] = k < MLP_IN ? bf16_bits(P[OFF_W1 + h * MLP_IN + k]) : bf16_bits(0.0f);
    }
    if (i < 2 * 4 * 32 * 16) {
        const int k = i & 15, row = (i >> 4) & 31, c = (i >> 9) & 3, mb = i >> 11;
        const int hk = mlp_kperm(c, k);
        W->w2[mb][c][row][k] = bf16_bits(P[OFF_W2 + (mb * 32 + row) * MLP_H + hk]);
        W->w2t[mb][c][row][k] = bf16_bits(P[OFF_W2 + hk * MLP_H + (mb * 32 + row)]);
    }
    if (i < MLP_H) {
        W->b1[i] = P[OFF_B1 + i];
        W->b2[i] = P[OFF_B2 + i];
        W->w3[i] = P[OFF_W3 + i];
    }
    if (i == 0) W->b3 = P[OFF_B3];
}

__device__ __forceinline__ void load_weights_lds(MlpWeights& dst, const MlpWeights* __restrict__ src) {
    const int nwords = sizeof(MlpWeights) / 4;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const MlpWeights* __restrict__ Wg, const float* __restrict__ x,
                                                          float* __restrict__ y, int32_t B) {
    __shared__ MlpWeights W;
    load_weights_lds(W, Wg);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < B;
    float f[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) f[k] = ok ? x[(size_t)i * MLP_IN + k] : 0.0f;
    const float out = mlp_eval(W, f, nullptr);
    if (ok) y[i] = out;
}

// one wave (64 samples) per workgroup
struct GradTiles {
    float dz2[MLP_H][65];   // [o][sample]
    float h1[MLP_H][65];    // [h][sample]
    float dz1[MLP_H][65];   // [h][sample]
    float x[MLP_IN][65];    // [k][sample]
    float dy[64];
};

// Each workgroup writes its partial gradient (and loss) to its own row of
// `part` ([blocks][MLP_NPARAM + 1]); mlp_reduce_kernel sums the rows in a
// fixed order, so gradients are reproducible bit for bit.
__global__ void __launch_bounds__(64) mlp_grads_kernel(const MlpWeights* __restrict__ Wg, const float* __restrict__ x,
                                                       const float* __restrict__ t, int32_t B,
                                                       float* __restrict__ part) {
    float* grad = part + (size_t)blockIdx.x * (MLP_NPARAM + 1);
    float* loss = grad + MLP_NPARAM;
    __shared__ MlpWeights W;
    __shared__ GradTiles T;
    load_weights_lds(W, Wg);
    const int l = threadIdx.x;
    const int hi = l >> 5, r32 = l & 31;
    const int i = blockIdx.x * 64 + l;
    const bool ok = i < B;
    float f[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) f[k] = ok ? x[(size_t)i * MLP_IN + k] : 0.0f;
    MlpActs A;
    const float y = mlp_eval(W, f, &A);
    const float d = ok ? (y - t[i]) : 0.0f;
    const float dy = 2.0f * d / (float)B;
    // loss partial
    float sq = d * d / (float)B;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (l == 0) *loss = sq;
    // dy of the samples of column blocks 0 and 1
    const float dy_other = __shfl_xor(dy, 32);
    const float dyb[2] = {hi ? dy_other : dy, hi ? dy : dy_other};
    // dz2 (register layout of z2) and the tiles for the weight gradients
    floatx16 dz2[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int o = mb * 32 + blk_row(j, hi);
                const float g = A.z2[mb][nb][j] > 0.0f ? dyb[nb] * W.w3[o] : 0.0f;
                dz2[mb][nb][j] = g;
                T.dz2[o][nb * 32 + r32] = g;
                T.h1[o][nb * 32 + r32] = relu(A.z1[mb][nb][j]);
            }
    // dh1 = W2^T dz2 on the matrix cores; K order = dz2's register order
    floatx16 dz1[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = {};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bf16x8 a = load_bf16x8(&W.w2t[mb][c][r32][8 * hi]);
                bf16x8 b;
#pragma unroll
                for (int k = 0; k < 8; ++k) b[k] = (__bf16)dz2[c >> 1][nb][8 * (c & 1) + k];
                acc = mfma32(a, b, acc);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int h = mb * 32 + blk_row(j, hi);
                const float g = A.z1[mb][nb][j] > 0.0f ? acc[j] : 0.0f;
                dz1[mb][nb][j] = g;
                T.dz1[h][nb * 32 + r32] = g;
            }
        }
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) T.x[k][l] = f[k];
    T.dy[l] = dy;
    __syncthreads();
    // weight gradients on the matrix cores, contracting over the wave's 64
    // samples: dW2 = dz2 h1^T (64 x 64) and dW1 = dz1 x^T (64 x 7), BF16
    // operands and FP32 accumulation.  The A operand of an output row block
    // comes from that row's [row][sample] tile (lane l: row l % 32, samples
    // 8 (l / 32) .. + 8 of the K step), the B operand from the columns' tiles
    // likewise; output element j of lane l is (row blk_row(j), column l % 32).
    auto tile_bf16 = [&](const float* row, int s0) -> bf16x8 {
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (__bf16)row[s0 + k];
        return v;
    };
    const bf16x8 zero8 = {};
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = {};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int s0 = kc * 16 + 8 * hi;
                acc = mfma32(tile_bf16(T.dz2[mb * 32 + r32], s0), tile_bf16(T.h1[nb * 32 + r32], s0), acc);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                grad[OFF_W2 + (mb * 32 + blk_row(j, hi)) * MLP_H + nb * 32 + r32] = acc[j];
        }
        // dW1: the B operand's columns are the 7 features (columns 7..31 zero)
        floatx16 acc = {};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            const int s0 = kc * 16 + 8 * hi;
            const bf16x8 xb = tile_bf16(T.x[r32 < MLP_IN ? r32 : 0], s0);
            acc = mfma32(tile_bf16(T.dz1[mb * 32 + r32], s0), r32 < MLP_IN ? xb : zero8, acc);
        }
        if (r32 < MLP_IN) {
#pragma unroll
            for (int j = 0; j < 16; ++j) grad[OFF_W1 + (mb * 32 + blk_row(j, hi)) * MLP_IN + r32] = acc[j];
        }
    }
    // bias gradients: lane l sums row l of dz2 and dz1 over the samples (FP32)
    const int o = l;
    float gb2 = 0.0f, gb1 = 0.0f, gb3 = 0.0f;
    for (int s = 0; s < 64; ++s) {
        gb2 += T.dz2[o][s];
        gb1 += T.dz1[o][s];
    }
    // h2 = relu(z2) is not in the tiles: w3's gradient from dz2 / w3 is
    // ill-defined at w3 = 0, so it is accumulated from h2 directly below
    grad[OFF_B2 + o] = gb2;
    grad[OFF_B1 + o] = gb1;
    // w3 and b3: sum over the samples of dy * h2 (each lane has 32 hidden units of 2 samples)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            float v = 0.0f;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) v = fmaf(dyb[nb], relu(A.z2[mb][nb][j]), v);
            // reduce over the 32 lanes of this half (same hidden unit)
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (r32 == 0) grad[OFF_W3 + mb * 32 + blk_row(j, hi)] = v;
        }
    gb3 = dy;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gb3 += __shfl_xor(gb3, off);
    if (l == 0) grad[OFF_B3] = gb3;
}

__global__ void mlp_reduce_kernel(const float* __restrict__ part, int nblk, float* __restrict__ g,
                                  float* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > MLP_NPARAM) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * (MLP_NPARAM + 1) + i];
    if (i < MLP_NPARAM) g[i] = s;
    else *loss = s;
}

__global__ void mlp_adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void mlp_features_kernel(int32_t n, const float* __restrict__ par, const float* __restrict__ q,
                                    const float* __restrict__ R, const float* __restrict__ s_label, float bz,
                                    float* __restrict__ x, float* __restrict__ t, float* __restrict__ s_line) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* p = par + (size_t)i * 6;
    float sphi, cphi;
    sincosf(p[4], &sphi, &cphi);
    const float w = -q[i] * KAPPA_MLP * bz * p[3];
    float f[MLP_IN], sl;
    mlp_features_of(p[0], p[1], cphi, sphi, w, R[i], f, sl);
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) x[(size_t)i * MLP_IN + k] = f[k];
    if (s_line) s_line[i] = sl;
    if (t && s_label) t[i] = sl > 0.0f ? asinhf(MLP_TARGET_SCALE * (s_label[i] / sl - 1.0f)) : 0.0f;
}

hipError_t mlp_recast(const MlpDev& d, hipStream_t s) {
    hipLaunchKernelGGL(mlp_recast_kernel, dim3((2 * 4 * 32 * 16 + 255) / 256), dim3(256), 0, s, d.master, d.w);
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpDev& d, const float* x, float* y, int32_t B, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 255) / 256), dim3(256), 0, s, d.w, x, y, B);
    return hipGetLastError();
}

int mlp_grad_blocks(int32_t B) { return (B + 63) / 64; }

hipError_t mlp_grads(const MlpDev& d, const float* x, const float* t, int32_t B, hipStream_t s) {
    const int nblk = mlp_grad_blocks(B);
    hipLaunchKernelGGL(mlp_grads_kernel, dim3(nblk), dim3(64), 0, s, d.w, x, t, B, d.part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, s, d.part, nblk, d.grad,
                       d.loss);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpDev& d, float lr, int32_t step, hipStream_t s) {
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)step));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)step));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, d.master, d.m, d.v, d.grad,
                       lr, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_recast(d, s);
}

hipError_t mlp_features(int32_t n, const float* par, const float* q, const float* R, const float* s_label,
                        float bz, float* x, float* t, float* s_line, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_features_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, par, q, R, s_label, bz, x, t,
                       s_line);
    return hipGetLastError();
}

}  // namespace p2r
