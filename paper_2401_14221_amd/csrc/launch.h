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
};

hipError_t launch_fit(const Variant& v, const FitLaunch& a, const Params& P, hipStream_t s);

// Ragged path
struct RaggedLaunch {
    int32_t n;                 // tracks
    int64_t H;                 // total surfaces
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
    // workspace (device)
    int32_t* counts;           // [lmax+2] histogram / offsets of surface counts
    int32_t* perm;             // [n] packed order -> track index
    int32_t* work;             // [1] work-queue counter
    float* trk_pack;           // [nb][28][W]
    float* hit_pack;           // [nb][lmax][11][W]  (9 hit values + surface value + type)
    int32_t* blk_len;          // [nb] surfaces of the longest track of each block
    int32_t nb;
    int32_t lmax;
    int32_t grid;              // persistent grid size
};

hipError_t launch_ragged(const Variant& v, const RaggedLaunch& a, const Params& P, hipStream_t s);
int ragged_lmax_limit();

}  // namespace p2r
