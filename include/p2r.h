/*
 * p2r.h -- C ABI of libp2r.so, the MI355X (gfx950) track-fit hot path.
 *
 * The library runs the per-track loop of the p2r / p2z mini-apps (paper,
 * Section 2): for every track and every detector surface in order, propagate
 * the helix state (x, y, z, 1/pT, phi, theta; charge q separate) to the
 * surface in a uniform field B z-hat, transport the 6x6 covariance with the
 * Jacobian (C' = J C J^T), and Kalman-update with the surface's 3D hit
 * (innovation covariance S, gain, state and Joseph-form covariance update,
 * chi2).  One GPU lane handles one track; the arithmetic is FP32 with an FP64
 * 3x3 inversion when the FP32 positive-definiteness test of S fails.
 *
 * Units: cm, GeV, tesla, radians.  Curvature omega = -q * 2.99792458e-3 * B / pT
 * [1/cm]; positive tracks turn clockwise seen from +z.  Path lengths are
 * transverse arc lengths.  Covariances are packed lower triangles,
 * row-major: element (i, j), j <= i, at index i(i+1)/2 + j.
 *
 * Conventions for every call below:
 *  - Buffer pointers are DEVICE pointers owned by the caller unless stated
 *    otherwise; the library never frees or keeps them past the call.
 *  - Calls are asynchronous on the caller's HIP stream (passed as void*,
 *    a hipStream_t; NULL = the default stream).  No implicit synchronisation.
 *  - Return 0 on success or a negative P2R_E* code; p2r_last_error() gives a
 *    thread-local message.  Argument errors are detected on the host and
 *    never launch anything.
 *  - Per-track numerical problems are never errors: they are reported in the
 *    status word (P2R_ST_* bits below) and the track keeps its last state.
 *  - The library allocates device memory only in p2r_ctx_create,
 *    p2r_mlp_create and, once per shape, in fit_tracks_batched (its
 *    workspace and graph); everything is released by the matching destroy.
 *
 * Status word per track: bits 0..7 flags, bits 8..15 the number of surfaces
 * whose update was applied, bit 31 set when the track was processed.
 */
#ifndef P2R_H
#define P2R_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define P2R_OK 0
#define P2R_EINVAL (-1)    /* bad argument (null pointer, negative size, ...) */
#define P2R_ELAYOUT (-2)   /* layout width not supported / misaligned buffer */
#define P2R_EHIP (-3)      /* a HIP runtime call failed (message has the HIP error) */
#define P2R_ENOTUNED (-4)  /* no tuned variant and tuning was required */

/* status flags */
#define P2R_ST_NO_CROSSING (1u << 0)   /* surface not reachable: layer skipped */
#define P2R_ST_NEWTON_FAIL (1u << 1)   /* helix-to-r iteration did not converge: layer skipped */
#define P2R_ST_FP64_FALLBACK (1u << 2) /* FP32 PD test of S failed, FP64 inversion used */
#define P2R_ST_S_NOT_PD (1u << 3)      /* S not PD even in FP64: update skipped, state propagated */
#define P2R_ST_BAD_INPUT (1u << 4)     /* non-finite input, 1/pT <= 0 or theta not in (0, pi): not processed */
#define P2R_ST_ML_REJECTED (1u << 5)   /* learned path-length proposal rejected, plain start used */
#define P2R_ST_HIT_MISSING (1u << 6)   /* non-finite hit position: layer skipped */
#define P2R_ST_CHI2_CUT (1u << 7)      /* chi2 above the cut: update skipped, state propagated */
#define P2R_ST_DONE (1u << 31)
#define P2R_ST_NUSED(st) (((st) >> 8) & 0xffu)

/* Track record: 28 floats = 6 parameters, 21 packed covariance values, and
 * the charge (+1.0f or -1.0f).  In the AoSoA layouts field f of the track in
 * lane l of block b is at trk[(b * 28 + f) * W + l].  Hit record: 9 floats =
 * position (x, y, z) and the packed 3x3 covariance (xx, yx, yy, zx, zy, zz). */
#define P2R_TRACK_FIELDS 28
#define P2R_HIT_FIELDS 9

typedef struct p2r_ctx p2r_ctx; /* opaque: device, tuned variants, workspace, graphs */

/* Fit options.  p2r_opts_default() fills: bz 3.8 T, newton_tol 1e-6 cm,
 * 8 iterations, chi2 cut off, FP64 fallback on, width 0 (tuned/default),
 * no MLP. */
typedef struct {
    float bz_tesla;          /* field along +z */
    float newton_tol_cm;     /* |r(s) - R| tolerance, raised to 2 ulp(R) */
    int32_t newton_max_iter; /* helix evaluations before NEWTON_FAIL */
    float chi2_cut;          /* <= 0: off; else skip updates with chi2 > cut */
    int32_t fp64_fallback;   /* 1: FP64 inversion when the FP32 PD test fails; 0: skip the update
                                instead; 2: always invert S in FP64 (testing) */
    int32_t width;           /* AoSoA width for p2r: 0 = context's tuned width, or 32/64/128/256 */
    const void* mlp;         /* NULL: plain start; else a p2r_mlp handle (learned start, p2r only) */
} p2r_opts;

void p2r_opts_default(p2r_opts* o);
const char* p2r_last_error(void);
const char* p2r_version(void);

/* Create a context on HIP device `device`.  tune_cache_path (nullable, host
 * string) names a JSON file the autotuner reads and writes. */
int p2r_ctx_create(p2r_ctx** out, int device, const char* tune_cache_path);
void p2r_ctx_destroy(p2r_ctx* ctx);

/* Width the context uses for `which` (0 p2r, 1 p2z, 2 ragged). */
int p2r_layout_width(p2r_ctx* ctx, int which, int32_t* W_out);

/* p2r (paper Section 2, propagation to fixed-r barrel layers).
 * n_tracks tracks, n_layers cylinders of radius layer_r[l] (device,
 * increasing outward is typical but not required).  Layout (AoSoA width W =
 * opts->width or the context's width):
 *   trk_in, trk_out: [ceil(n_tracks/W)][28][W] floats
 *   hits:            [ceil(n_tracks/W)][n_layers][9][W] floats
 *   chi2_out: [n_tracks] summed chi2; status: [n_tracks] status words.
 * Lanes past n_tracks in the last block are neither read nor written.
 * Each layer: crossing by Newton iteration on r(s) - R from the straight-line
 * path (or the learned proposal), then the update. */
int p2r_propagate_update(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                         const float* layer_r, const float* trk_in, const float* hits,
                         float* trk_out, float* chi2_out, uint32_t* status, void* stream);

/* p2z (paper Section 2, propagation to fixed-z disks).  Disk l is the plane
 * z = +layer_z[l] for tracks whose input theta < float(pi/2), else
 * z = -layer_z[l].  Path length s = (Z - z) tan(theta) in closed form.
 * Layout (width 64, layer-outer hits):
 *   trk_in, trk_out: [ceil(n_tracks/64)][28][64] floats
 *   hits:            [n_layers][ceil(n_tracks/64)][9][64] floats */
int p2z_propagate_update(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                         const float* layer_z, const float* trk_in, const float* hits,
                         float* trk_out, float* chi2_out, uint32_t* status, void* stream);

/* Ragged batched fit: every track has its own ordered list of surfaces
 * (CSR), each a cylinder (surf_type 0, surf_val = radius) or a plane
 * (surf_type 1, surf_val = signed z), and one 3D hit per surface.
 *   offsets [n_tracks+1] (int64, offsets[0] = 0), surf_type [H] (uint8),
 *   surf_val [H], hit_pos [H][3], hit_cov [H][6] (packed), par_in [n][6],
 *   cov_in [n][21], q [n] (int8 +-1); outputs par_out [n][6],
 *   cov_out [n][21], chi2_out [n], status [n].
 * Tracks are packed (sorted by surface count) into the AoSoA layout by a
 * device kernel and fitted by one persistent kernel that takes blocks of
 * tracks from an atomic work queue; the three steps run as one HIP graph,
 * captured on the first call for a given (n_tracks, total surfaces) and
 * replayed afterwards.  The packing workspace lives in the context and is
 * reused: calls on one context must not overlap. */
int fit_tracks_batched(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, const int64_t* offsets,
                       const uint8_t* surf_type, const float* surf_val, const float* hit_pos,
                       const float* hit_cov, const float* par_in, const float* cov_in, const int8_t* q,
                       float* par_out, float* cov_out, float* chi2_out, uint32_t* status, void* stream);

/* Autotune `which` (0 p2r, 1 p2z, 2 ragged) on synthetic tracks of this
 * shape: times every compiled variant (width, waves per SIMD, layer-loop
 * unroll) with HIP events, keeps the fastest in the context and writes the
 * cache file if the context has one.  Synchronises the stream. */
int p2r_autotune(p2r_ctx* ctx, int which, int32_t n_tracks, int32_t n_layers, void* stream);

/* Description of the variant in use for `which` (host string owned by ctx). */
const char* p2r_variant_name(p2r_ctx* ctx, int which);

#ifdef __cplusplus
}
#endif
#endif /* P2R_H */
