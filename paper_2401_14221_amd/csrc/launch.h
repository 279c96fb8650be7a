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

const std::vector<Variant>& variants();

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
// bin), their hits packed per block of RAG_W sorted tracks into
// [layer][RAG_FIELDS][RAG_W] rows, then the fit kernel over the blocks.
constexpr int RAG_W = 64;
constexpr int RAG_ETA_BINS = 8;
constexpr int RAG_FIELDS = 11;      // surface type, surface value, hit (3), hit covariance (6)
constexpr int RAG_TPB = 1024;       // tracks per workgroup in the sort kernels

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
    int64_t* run;              // [n] sorted position -> the track's first hit | surface count << 56
                               //     (RAG_RUN_SHIFT), or -1 for a track in the invalid bucket
    int32_t* blk_off;          // [nb + 1] first packed layer row of each block
    float* packed;             // [packed_cap][RAG_FIELDS][RAG_W] hits of the sorted blocks
    int64_t packed_cap;        // layer rows available in packed
    int32_t nkeys;
    int32_t nb;                // blocks of RAG_W sorted tracks
    int32_t grid;              // workgroups of the persistent variant (one wave each)
};

// Layer rows the packed hits of n tracks with n_hits surfaces in total can
// need when the CSR ranges do not overlap (blocks that would not fit are
// reported as BAD_INPUT by the fit).
int64_t ragged_packed_rows(int64_t n_hits, int lmax);
constexpr int RAG_RUN_SHIFT = 56;
int ragged_nkeys(int lmax);
hipError_t launch_ragged(const Variant& v, const RaggedLaunch& a, const Params& P, hipStream_t s);

}  // namespace p2r
