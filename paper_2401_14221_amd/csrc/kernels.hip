// Fit kernels for gfx950: one lane per track, the whole layer loop in one
// launch (the paper's single fused kernel, Section 2).  Track records are
// read once, coalesced, into registers; hits stream in per layer, the next
// layer's hit prefetched while the current layer is computed; results are
// written once at the end.
#include "launch.h"
#include "mlp_dev.h"
#include "track_math.h"

namespace p2r {

template <typename T>
__device__ __forceinline__ void load_track(const float* __restrict__ t, int W, StateT<T>& st) {
#pragma unroll
    for (int f = 0; f < 6; ++f) st.p[f] = (T)t[f * W];
#pragma unroll
    for (int f = 0; f < 21; ++f) st.c[f] = (T)t[(6 + f) * W];
    st.q = (T)t[27 * W];
}

// results are stored in FP32 whatever the arithmetic type
template <typename T>
__device__ __forceinline__ void store_track(float* __restrict__ t, int W, const StateT<T>& st) {
#pragma unroll
    for (int f = 0; f < 6; ++f) t[f * W] = (float)st.p[f];
#pragma unroll
    for (int f = 0; f < 21; ++f) t[(6 + f) * W] = (float)st.c[f];
    t[27 * W] = (float)st.q;
}

// Sums the lanes' helix evaluations into *evals.  Every lane of the wave
// must reach this call (the cross-lane reduction reads all 64 lanes), so a
// kernel that counts keeps its lanes past n in the loop, shadowing the last
// track with a count of zero.
__device__ __forceinline__ void count_evals(unsigned long long* evals, int iters) {
    if (!evals) return;
    unsigned long long v = (unsigned long long)iters;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (__lane_id() == 0) atomicAdd(evals, v);
}

// The next layer's surface value, loaded with the next layer's hit.  The
// table is read through a vector load (the kernel's stores could alias it as
// far as the compiler knows), and vector loads land in order: one issued
// after the hit prefetch and used in the current layer would make the layer
// wait for the whole prefetch.  Loaded a layer ahead, it is needed only when
// the prefetch is.
__device__ __forceinline__ float next_surface(const float* surf, int ly) { return surf[ly]; }

// p2r: hits [block][layer][9][W].  LEARNED: the path-length MLP proposes the
// start of every helix-to-cylinder solve; the whole wave evaluates it on the
// matrix cores, so every lane stays in the layer loop (lanes past n shadow
// the last track and write nothing).
template <int W, int UNROLL, bool LEARNED, typename T = float, bool U2D = false>
__device__ __forceinline__ void p2r_body(const FitLaunch& a, const Params& P, MlpWeights* Wl) {
    if (LEARNED) {
        const uint32_t* s = reinterpret_cast<const uint32_t*>(a.mlp);
        uint32_t* d = reinterpret_cast<uint32_t*>(Wl);
        for (int i = threadIdx.x; i < (int)(sizeof(MlpWeights) / 4); i += blockDim.x) d[i] = s[i];
        __syncthreads();
    }
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = gid < a.n;
    // lanes past n leave at once unless the wave must stay whole: the learned
    // start evaluates the network over the whole wave, and the evaluation
    // count is a reduction over all 64 lanes
    if (!LEARNED && !active && !a.evals) return;
    const int g = active ? gid : a.n - 1;
    const int b = g / W, l = g % W;
    const float* tin = a.trk_in + (size_t)b * (28 * W) + l;
    StateT<T> st;
    load_track(tin, W, st);
    uint32_t flags = 0;
    int nused = 0, evals = 0;
    T chi2 = 0;
    const bool bad = bad_input(st);
    if (bad) flags = ST_BAD_INPUT;
    if (!bad || LEARNED) {
        const float* hb = a.hits + (size_t)b * ((size_t)a.L * 9 * W) + l;
        // with no layers the hit stream is the track records (launch_fit), so
        // this first prefetch stays inside a buffer; its values are unused
        float hm[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) hm[k] = hb[k * W];
        // the layer radius travels with the prefetched hit (see next_surface)
        float rn = a.L > 0 ? a.surf[0] : 0.0f;
#pragma unroll UNROLL
        for (int ly = 0; ly < a.L; ++ly) {
            const T m[3] = {hm[0], hm[1], hm[2]};
            const T V[6] = {hm[3], hm[4], hm[5], hm[6], hm[7], hm[8]};
            const T R = rn;
            if (ly + 1 < a.L) {
                const float* hn = hb + (size_t)(ly + 1) * (9 * W);
#pragma unroll
                for (int k = 0; k < 9; ++k) hm[k] = hn[k * W];
                rn = next_surface(a.surf, ly + 1);
            }
            T s_start = NAN;
            if (LEARNED) {
                float sphi, cphi;
                sincosf((float)st.p[4], &sphi, &cphi);
                const float w = (float)(-st.q * KAPPA * P.bz * st.p[3]);
                float feat[MLP_IN], sl;
                const bool ok = mlp_features_of((float)st.p[0], (float)st.p[1], cphi, sphi, w, (float)R, feat, sl);
                // an offset the compiler cannot see through keeps the weight
                // reads in LDS inside the loop; hoisted, they would pin ~130
                // registers for the whole fit
                int zoff = 0;
                asm volatile("" : "+s"(zoff));
                const MlpWeights* Wv = reinterpret_cast<const MlpWeights*>(reinterpret_cast<const char*>(Wl) + zoff);
                const float yv = mlp_infer(*Wv, feat);            // whole wave
                if (ok && !bad && finite3(m)) s_start = sl * (1.0f + sinhf(fminf(fmaxf(yv, -8.0f), 8.0f)) * (1.0f / MLP_TARGET_SCALE));
            }
            if (!bad) {
                T c2 = 0;
                StepOut o = step_cylinder<T, U2D>(st, R, m, V, P, c2, newton_tol(P.tol, R), s_start, T(MLP_ACCEPT_CM));
                flags |= o.flags;
                evals += o.iters;
                if (o.updated) { ++nused; chi2 += c2; }
            }
        }
    }
    count_evals(a.evals, active ? evals : 0);
    if (!active) return;
    finalise(st);
    store_track(a.trk_out + (size_t)b * (28 * W) + l, W, st);
    a.chi2[gid] = (float)chi2;
    a.status[gid] = flags | ST_DONE | nused_field(nused);
}

// p2z: W = 64, hits [layer][block][9][64]; disk sign from the input theta
template <int UNROLL, typename T = float>
__device__ __forceinline__ void p2z_body(const FitLaunch& a, const Params& P) {
    constexpr int W = 64;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.n) return;
    const int b = gid / W, l = gid % W;
    const int nb = (a.n + W - 1) / W;
    const float* tin = a.trk_in + (size_t)b * (28 * W) + l;
    StateT<T> st;
    load_track(tin, W, st);
    uint32_t flags = 0;
    int nused = 0;
    T chi2 = 0;
    if (bad_input(st)) {
        flags = ST_BAD_INPUT;
    } else {
        const T zsign = (float)st.p[5] < HALF_PI_F ? T(1) : T(-1);
        const size_t lstride = (size_t)nb * (9 * W);
        const float* hb = a.hits + (size_t)b * (9 * W) + l;
        float hm[9];                      // (no layers: see p2r_body)
#pragma unroll
        for (int k = 0; k < 9; ++k) hm[k] = hb[k * W];
        float zn = a.L > 0 ? a.surf[0] : 0.0f;
#pragma unroll UNROLL
        for (int ly = 0; ly < a.L; ++ly) {
            const T m[3] = {hm[0], hm[1], hm[2]};
            const T V[6] = {hm[3], hm[4], hm[5], hm[6], hm[7], hm[8]};
            const T Z = zn;
            if (ly + 1 < a.L) {
                const float* hn = hb + (size_t)(ly + 1) * lstride;
#pragma unroll
                for (int k = 0; k < 9; ++k) hm[k] = hn[k * W];
                zn = next_surface(a.surf, ly + 1);
            }
            T c2 = 0;
            StepOut o = step_plane<T>(st, zsign * Z, m, V, P, c2);
            flags |= o.flags;
            if (o.updated) { ++nused; chi2 += c2; }
        }
    }
    finalise(st);
    store_track(a.trk_out + (size_t)b * (28 * W) + l, W, st);
    a.chi2[gid] = (float)chi2;
    a.status[gid] = flags | ST_DONE | nused_field(nused);
}

#define P2R_KERNEL(W, WPE, U)                                                              \
    __global__ void __attribute__((amdgpu_flat_work_group_size(256, 256),                \
                                   amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))               \
    p2r_w##W##_e##WPE##_u##U(FitLaunch a, Params P) { p2r_body<W, U, false>(a, P, nullptr); }

#define P2R_LEARNED_KERNEL(W, WPE, U)                                                      \
    __global__ void __attribute__((amdgpu_flat_work_group_size(256, 256),                \
                                   amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))               \
    p2r_mlp_w##W##_e##WPE##_u##U(FitLaunch a, Params P) {                                 \
        __shared__ MlpWeights Wl;                                                          \
        p2r_body<W, U, true>(a, P, &Wl);                                                   \
    }

#define P2Z_KERNEL(WPE, U)                                                                 \
    __global__ void __attribute__((amdgpu_flat_work_group_size(256, 256),                \
                                   amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))               \
    p2z_w64_e##WPE##_u##U(FitLaunch a, Params P) { p2z_body<U>(a, P); }

P2R_KERNEL(32, 0, 1)
P2R_KERNEL(64, 0, 1)
P2R_KERNEL(128, 0, 1)
P2R_KERNEL(256, 0, 1)
P2R_KERNEL(64, 4, 1)
P2R_KERNEL(64, 5, 1)
P2R_KERNEL(64, 0, 2)
P2R_KERNEL(128, 4, 1)
P2R_KERNEL(256, 4, 1)
// Learned start: built for 3 waves per SIMD (168 registers, 16 bytes of
// spill).  Measured on the 960,000-track workload: the compiler's own
// choice, 196 registers (2 waves per SIMD), runs 14% slower; for 4 waves it
// spills ~140 bytes per lane in the layer loop and runs 44% slower.
P2R_LEARNED_KERNEL(64, 3, 1)
P2R_LEARNED_KERNEL(128, 3, 1)
P2R_LEARNED_KERNEL(256, 3, 1)
P2R_LEARNED_KERNEL(32, 3, 1)
// FP64 fits: every step in FP64 on the same FP32 inputs, results rounded to
// FP32 (a precision and throughput reference for the FP32 kernels).  Built
// for 2 waves per SIMD: the state in FP64 needs more than 256 registers, and
// spilling a few of them (tens of bytes per lane) costs less than running
// one wave per SIMD with nothing to hide its latencies.
#define P2R_F64_KERNEL(W)                                                                     \
    __global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2))) \
    p2r_f64_w##W(FitLaunch a, Params P) { p2r_body<W, 1, false, double>(a, P, nullptr); }
P2R_F64_KERNEL(32)
P2R_F64_KERNEL(64)
P2R_F64_KERNEL(128)
P2R_F64_KERNEL(256)
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2))) p2z_f64_w64(FitLaunch a, Params P) {
    p2z_body<1, double>(a, P);
}

// p2r with the update in the hit's (r-phi, z) frame.  Compiled for 4 waves
// per SIMD (128 VGPRs): the only values that go to scratch memory are the
// argument copies of the rare FP64 calls.
#define P2R_2D_KERNEL(W)                                                                  \
    __global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(4)))  \
    p2r_2d_w##W(FitLaunch a, Params P) { p2r_body<W, 1, false, float, true>(a, P, nullptr); }
P2R_2D_KERNEL(32)
P2R_2D_KERNEL(64)
P2R_2D_KERNEL(128)
P2R_2D_KERNEL(256)
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2))) p2r_f64_2d_w64(FitLaunch a, Params P) {
    p2r_body<64, 1, false, double, true>(a, P, nullptr);
}

P2Z_KERNEL(0, 1)
P2Z_KERNEL(4, 1)
P2Z_KERNEL(5, 1)
P2Z_KERNEL(0, 2)

#define VAR(WH, W, E, U, K) Variant{WH, W, E, U, #K, (const void*)&K, false, false, false}
#define VARL(W, E, U, K) Variant{0, W, E, U, #K, (const void*)&K, true, false, false}
#define VARD(WH, W, K) Variant{WH, W, 0, 1, #K, (const void*)&K, false, true, false}
#define VAR2(W, F64, K) Variant{0, W, 0, 1, #K, (const void*)&K, false, F64, true}

static std::vector<Variant> make_variants() {
    std::vector<Variant> v = {
        VAR(0, 64, 0, 1, p2r_w64_e0_u1),   // default p2r
        VAR(0, 32, 0, 1, p2r_w32_e0_u1),
        VAR(0, 128, 0, 1, p2r_w128_e0_u1),
        VAR(0, 256, 0, 1, p2r_w256_e0_u1),
        VAR(0, 64, 4, 1, p2r_w64_e4_u1),
        VAR(0, 64, 5, 1, p2r_w64_e5_u1),
        VAR(0, 64, 0, 2, p2r_w64_e0_u2),
        VAR(0, 128, 4, 1, p2r_w128_e4_u1),
        VAR(0, 256, 4, 1, p2r_w256_e4_u1),
        VAR(1, 64, 0, 1, p2z_w64_e0_u1),   // default p2z
        VAR(1, 64, 4, 1, p2z_w64_e4_u1),
        VAR(1, 64, 5, 1, p2z_w64_e5_u1),
        VAR(1, 64, 0, 2, p2z_w64_e0_u2),
        VAR2(64, false, p2r_2d_w64),       // update in the hit frame
        VAR2(32, false, p2r_2d_w32),
        VAR2(128, false, p2r_2d_w128),
        VAR2(256, false, p2r_2d_w256),
        VAR2(64, true, p2r_f64_2d_w64),
        VARD(0, 64, p2r_f64_w64),          // FP64 fits, one per width
        VARD(0, 32, p2r_f64_w32),
        VARD(0, 128, p2r_f64_w128),
        VARD(0, 256, p2r_f64_w256),
        VARD(1, 64, p2z_f64_w64),
        VARL(64, 3, 1, p2r_mlp_w64_e3_u1),     // learned start, one per width
        VARL(128, 3, 1, p2r_mlp_w128_e3_u1),
        VARL(256, 3, 1, p2r_mlp_w256_e3_u1),
        VARL(32, 3, 1, p2r_mlp_w32_e3_u1),
    };
    append_ragged_variants(v);
    return v;
}

const std::vector<Variant>& variants() {
    static const std::vector<Variant> v = make_variants();
    return v;
}

hipError_t launch_fit(const Variant& v, const FitLaunch& a, const Params& P, hipStream_t s) {
    const int threads = 256;
    const int blocks = (a.n + threads - 1) / threads;
    if (blocks == 0) return hipSuccess;
    FitLaunch aa = a;
    // The kernels prefetch the first layer's hit before their layer loop.
    // With no layers there may be no hit buffer: the prefetch then reads the
    // track records instead, and stays inside them -- p2r reads floats
    // l + k W (k < 9, l < W) and p2z reads 9 W b + k W + l of a record
    // buffer of 28 W floats per block -- and its values are never used.
    // (Guarding the prefetch with a branch on L instead made the learned
    // 256-wide kernel return wrong results with this compiler.)
    if (aa.L == 0) aa.hits = aa.trk_in;
    Params pp = P;
    void* args[] = {&aa, &pp};
    return hipLaunchKernel(v.fn, dim3(blocks), dim3(threads), args, 0, s);
}


// ----------------------------------------------------------- autotune data
// Plausible tracks for timing the variants: counter-hashed uniforms give
// pT in [0.5, 10] GeV, phi in (-pi, pi], eta in [-1.5, 1.5] (p2r) or
// |eta| in [1.7, 2.5] (p2z); the hits are the exact crossings of the
// unsmeared track (surfaces evenly spaced in r = 2.5..110 cm or
// |z| = 30..270 cm).
__global__ void synth_kernel(int which, int W, int32_t n, int32_t L, float* surf, float* trk, float* hits) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < L) {
        float t = L > 1 ? (float)gid / (float)(L - 1) : 0.0f;
        surf[gid] = which == 0 ? 2.5f + t * 107.5f : 30.0f + t * 240.0f;
    }
    if (gid >= n) return;
    const int b = gid / W, l = gid % W;
    const int nb = (n + W - 1) / W;
    float pt = 0.5f + 9.5f * hash_u01(gid, 1);
    float eta = which == 0 ? -1.5f + 3.0f * hash_u01(gid, 2)
                           : (1.7f + 0.8f * hash_u01(gid, 2)) * (hash_u01(gid, 5) < 0.5f ? -1.0f : 1.0f);
    float phi = -PI_F + TWO_PI_F * hash_u01(gid, 3);
    float q = hash_u01(gid, 4) < 0.5f ? -1.0f : 1.0f;
    State st;
    st.p[0] = 0.0f; st.p[1] = 0.0f; st.p[2] = 0.0f;
    st.p[3] = 1.0f / pt; st.p[4] = phi; st.p[5] = 2.0f * atanf(expf(-eta));
    for (int k = 0; k < 21; ++k) st.c[k] = 0.0f;
    st.c[I21(0, 0)] = 0.01f; st.c[I21(1, 1)] = 0.01f; st.c[I21(2, 2)] = 1.0f;
    st.c[I21(3, 3)] = 1e-4f; st.c[I21(4, 4)] = 1e-4f; st.c[I21(5, 5)] = 1e-4f;
    st.q = q;
    float* t = trk + (size_t)b * 28 * W + l;
    store_track(t, W, st);
    float x = 0.f, y = 0.f, z = 0.f, ph = phi;
    const float kq = -q * KAPPA * 3.8f;
    const float w = kq / pt;
    const float cot = 1.0f / tanf(st.p[5]);
    bool alive = true;
    for (int ly = 0; ly < L; ++ly) {
        float S = which == 0 ? 2.5f + (L > 1 ? (float)ly / (float)(L - 1) : 0.0f) * 107.5f
                             : 30.0f + (L > 1 ? (float)ly / (float)(L - 1) : 0.0f) * 240.0f;
        float m[3] = {NAN, NAN, NAN};
        float sphi, cphi;
        sincosf(ph, &sphi, &cphi);
        if (alive) {
            HelixT<float> h;
            float s = 0.0f;
            int it = 0;
            bool ok, lok;
            if (which == 0) {
                ok = cylinder_reachable(x, y, cphi, sphi, w, S) &&
                     newton_cylinder(x, y, cphi, sphi, w, S, newton_tol(1e-6f, S), 16,
                                     line_path(x, y, cphi, sphi, S, &lok), s, h, it);
            } else {
                float Z = eta > 0 ? S : -S;
                s = (Z - z) / cot;
                ok = s > 0.0f;
                if (ok) helix_at(x, y, cphi, sphi, w, s, h);
            }
            if (ok) {
                x = h.x; y = h.y; z = which == 0 ? z + s * cot : (eta > 0 ? S : -S);
                ph = ph + 2.0f * h.u;
                m[0] = x; m[1] = y; m[2] = z;
            } else {
                alive = false;
            }
        }
        float* hp = which == 0 ? hits + ((size_t)b * L + ly) * 9 * W + l
                               : hits + ((size_t)ly * nb + b) * 9 * W + l;
        const float V[6] = {1e-4f, 0.0f, 1e-4f, 0.0f, 0.0f, which == 0 ? 1e-2f : 1e-4f};
        for (int k = 0; k < 3; ++k) hp[k * W] = m[k];
        for (int k = 0; k < 6; ++k) hp[(3 + k) * W] = V[k];
    }
}

hipError_t launch_synth(int which, int W, int32_t n, int32_t L, float* surf, float* trk, float* hits,
                        hipStream_t s) {
    int m = n > L ? n : L;
    int blocks = (m + 255) / 256;
    hipLaunchKernelGGL(synth_kernel, dim3(blocks), dim3(256), 0, s, which, W, n, L, surf, trk, hits);
    return hipGetLastError();
}

}  // namespace p2r
