// Internal launch interface between the C ABI (capi.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace p2r {

struct Params;

// A compiled variant of a fit kernel.
struct Variant {
    int which;        // 0 p2r, 1 p2z, 2 ragged
    int width;        // AoSoA width W
    int waves_per_eu; // occupancy target the register budget is compiled for (0 = compiler's)
    int unroll;       // layer-loop unroll
    const char* name;
    const void* fn;   // kernel symbol
    bool learned;     // p2r with the MLP start
    bool fp64;        // every step in FP64 (FP32 inputs and results)
    bool upd2d;       // cylinders updated in the hit's (r-phi, z) frame
    bool per_block = false;   // ragged: one workgroup per block instead of the persistent work queue
};

// Counter-hashed uniform in [0, 1) for the autotuner's synthetic tracks
// (host and device compute the same values).
__host__ __device__ __forceinline__ float hash_u01(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
    return (h >> 8) * (1.0f / 16777216.0f);
}

const std::vector<Variant>& variants();
void append_ragged_variants(std::vector<Variant>& v);   // ragged.hip

struct FitLaunch {
    int32_t n, L;
    const float* surf;        // radii or |z|
    const float* trk_in;
    const float* hits;
    float* trk_out;
    float* chi2;
    uint32_t* status;
    const void* mlp;          // device MLP weights block (learned start) or null
    unsigned long long* evals;  // nullable: total helix evaluations (diagnostics)
};

hipError_t launch_fit(const Variant& v, const FitLaunch& a, const Params& P, hipStream_t s);

// Ragged path: tracks counting-sorted by (surface count descending, |eta|
// bin), then a fit kernel with one wave per block of RAG_W sorted tracks that
// stages the block's hits through LDS.
constexpr int RAG_W = 64;
constexpr int RAG_ETA_BINS = 8;
constexpr int RAG_FIELDS = 11;      // surface type, surface value, hit (3), hit covariance (6)
// Tracks per workgroup in the sort kernels.  Each workgroup ends with one
// global atomic per key it holds, and the atomics on one key serialise, so
// fewer, larger workgroups sort faster: at 10^6 tracks the histogram and
// scatter take 25 + 33 us with 1024 tracks per workgroup, 19 + 20 us with
// 4096 (245 workgroups, 16 tracks per thread).
constexpr int RAG_TPB = 4096;
constexpr int RAG_LSTRIDE = RAG_W + 1;  // floats per staged LDS row (one pad float)

struct RaggedLaunch {
    int32_t n;                 // tracks
    int32_t lmax;              // largest surface count a track may have
    int64_t n_hits;            // surfaces in total (bound of every CSR range)
    const int64_t* offsets;
    const uint8_t* stype;
    const float* sval;
    const float* hpos;
    const float* hcov;
    const float* par_in;
    const float* cov_in;
    const int8_t* q;
    float* par_out;
    float* cov_out;
    float* chi2;
    uint32_t* status;
    // workspace (device, owned by the context)
    int32_t* hist;             // [nkeys] tracks per sort key
    int32_t* base;             // [nkeys] first sorted position of each key, then scatter cursors
    int32_t* work;             // [1] work-queue counter
    int32_t* perm;             // [n] sorted position -> track index
    int32_t* keys;             // [n] sort key of every track
    int64_t* run;              // [n] sorted position -> the track's first hit | surface count << 48
                               //     (RAG_RUN_SHIFT), or -1 for a track in the invalid bucket
    int32_t nkeys;
    int32_t nb;                // blocks of RAG_W sorted tracks
    int32_t grid;              // workgroups of the persistent variant (one wave each)
};

// The first hit takes the low 48 bits (n_hits < 2^32), the surface count
// (0..255) the bits above, so that every valid run is non-negative and -1
// stays free for the invalid bucket (with the count at bit 56, counts of 128
// and more would set the sign bit and read as invalid).
constexpr int RAG_RUN_SHIFT = 48;
int ragged_nkeys(int lmax);
hipError_t launch_ragged(const Variant& v, const RaggedLaunch& a, const Params& P, hipStream_t s);

// Autotuner input for the ragged fit: the surface count of synthetic track t
// (5 .. lmax, or lmax when lmax < 5), and a kernel that fills each track's
// start (the origin, initial covariance of the fit workloads) and its CSR
// run of surfaces and exact hits.
__host__ __device__ __forceinline__ int ragged_synth_count(int32_t t, int lmax) {
    if (lmax < 5) return lmax;
    const int L = 5 + (int)(hash_u01((uint32_t)t, 11) * (float)(lmax - 4));
    return L > lmax ? lmax : L;
}
hipError_t launch_ragged_synth(int32_t n, int lmax, const int64_t* offsets, uint8_t* stype, float* sval,
                               float* hpos, float* hcov, float* par, float* cov, int8_t* q, hipStream_t s);

}  // namespace p2r
