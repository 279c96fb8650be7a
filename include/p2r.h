/*
 * p2r.h -- C ABI of libp2r.so, the MI355X (gfx950) track-fit hot path.
 *
 * The library runs the per-track loop of the p2r / p2z mini-apps (paper,
 * Section 2): for every track and every detector surface in order, propagate
 * the helix state (x, y, z, 1/pT, phi, theta; charge q separate) to the
 * surface in a uniform field B z-hat, transport the 6x6 covariance with the
 * Jacobian (C' = J C J^T), and Kalman-update with the surface's 3D hit
 * (innovation covariance S, gain, state and Joseph-form covariance update,
 * chi2 with 3 degrees of freedom).  The update is computed in the surface
 * frame of the crossing point: the transported position covariance has the
 * surface normal as a null direction, so the 3x3 update equals a 2x2 one with
 * the hit covariance and residual corrected for their normal component (a
 * Schur complement) plus the normal residual's chi2 term.  One GPU lane
 * handles one track; the arithmetic is FP32 with a compensated (two-part)
 * state, and the update is taken to FP64 when the FP32 positive-definiteness
 * test fails.
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
 *  - The library allocates device memory only in its sizing calls:
 *    p2r_ctx_reserve (the ragged workspace), p2r_ctx_reserve_host (the host
 *    pipeline's staging), p2r_mlp_create and p2r_mlp_reserve (weights,
 *    optimiser state, gradient partials), and p2r_autotune (temporaries).
 *    The fit, pipeline and training calls allocate nothing; a call that needs
 *    more workspace than was reserved returns P2R_ENOSPACE before launching.
 *    Everything is released by the matching destroy.
 *
 * Status word per track: bits 0..7 flags, bits 8..15 the number of surfaces
 * whose update was applied (saturating at 255), bit 31 set when the track
 * was processed.
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
#define P2R_ENOSPACE (-5)  /* the workspace reserved in the context is too small for this call */

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
/* Largest n_hits of one fit_tracks_batched call (the ragged fit addresses
 * its CSR arrays with 32-bit byte offsets: 24 * n_hits < 2^32). */
#define P2R_MAX_HITS 178956970LL
/* Limits of fit_tracks_batched_noalloc: tracks per call, and the bytes of
 * device memory its scratch array holds on every GPU the library runs on. */
#define P2R_NOALLOC_MAX_TRACKS 1048576
#define P2R_NOALLOC_SCRATCH_BYTES 16794368ULL

typedef struct p2r_ctx p2r_ctx; /* opaque: device, tuned variants, workspace, graphs */

/* Fit options.  p2r_opts_default() fills: bz 3.8 T, newton_tol 1e-6 cm,
 * 8 iterations, chi2 cut off, FP64 fallback 3, width 0 (tuned/default),
 * no MLP, graphs on, straight-line start, FP32 arithmetic. */
typedef struct {
    float bz_tesla;          /* field along +z */
    float newton_tol_cm;     /* |r(s) - R| tolerance, raised to 2 ulp(R) */
    int32_t newton_max_iter; /* helix evaluations before NEWTON_FAIL */
    float chi2_cut;          /* <= 0: off; else skip updates with chi2 > cut */
    int32_t fp64_fallback;   /* when the FP32 PD test (on the pivots of the surface-frame 2x2 S,
                                and V_nn > 0) fails: 3 = the whole 3x3 update (inverse, gain,
                                Joseph covariance) in FP64; 1 = only the 2x2 inverse in FP64;
                                0 = skip the update; 2 = the FP64 update for every surface
                                (testing) */
    int32_t width;           /* AoSoA width for p2r: 0 = context's tuned width, or 32/64/128/256 */
    const void* mlp;         /* NULL: plain start; else a p2r_mlp handle (learned start, p2r only) */
    int32_t use_graph;       /* fit_tracks_batched: 1 = capture once per shape and replay a HIP
                                graph (needs a non-NULL stream); 0 = launch the kernels directly */
    unsigned long long* helix_evals; /* nullable device counter: p2r adds the number of helix
                                evaluations of its cylinder solves (diagnostics) */
    int32_t cyl_start;       /* start of the helix-to-cylinder Newton iteration without an MLP:
                                0 = straight-line path (plain), 1 = closed-form FP32 crossing
                                (t = tan(omega s / 2) quadratic), which Newton then only checks */
    int32_t fp64;            /* 0 = FP32 arithmetic (default); 1 = every step in FP64 on the same
                                FP32 inputs, results rounded to FP32 (a precision reference; the
                                Newton tolerance becomes 1e-3 newton_tol_cm, the PD test the
                                FP64 one; not with an MLP) */
    int32_t update_2d;       /* cylinders: 0 = update with the 3D hit in global x, y, z (default);
                                1 = update in the hit's (r-phi, z) frame, 2 measured coordinates
                                (u = -s x + c y, z with (c, s) the hit's azimuth, V2 = R V R^T),
                                chi2 with 2 degrees of freedom.  Planes are unaffected: there the
                                3D update already equals the 2D one (the z residual is 0). */
} p2r_opts;

void p2r_opts_default(p2r_opts* o);
const char* p2r_last_error(void);
const char* p2r_version(void);

/* Create a context on HIP device `device`.  tune_cache_path (nullable, host
 * string) names a JSON file the autotuner reads and writes. */
int p2r_ctx_create(p2r_ctx** out, int device, const char* tune_cache_path);
void p2r_ctx_destroy(p2r_ctx* ctx);

/* Size the context's workspace for fit_tracks_batched calls of up to
 * max_tracks tracks with max_surfaces (0..255) surfaces per track: the sort
 * arrays (16 B per track) and the sort-key histograms (8 B per key, 8 keys
 * per surface count).  Grow-only; a call that grows the workspace frees the
 * old one (no ragged fit of this context may be in flight) and drops the
 * captured graph.  Synchronous. */
int p2r_ctx_reserve(p2r_ctx* ctx, int32_t max_tracks, int32_t max_surfaces);

/* Number of device allocations the library has made in this process (all
 * contexts and MLPs): a diagnostic for callers that must not allocate in
 * their timed or captured work. */
unsigned long long p2r_device_allocations(void);

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

/* Transfer-inclusive fits of host-resident tracks (the paper's p2z timing
 * includes the host-device copies, Section 4).  Same layouts, options and
 * per-track semantics as p2r_propagate_update / p2z_propagate_update, but
 * every array, layer_r / layer_z included, is in HOST memory.  The tracks go
 * in chunks of chunk_tracks (rounded up to whole blocks; 0 = 131072): each
 * chunk is copied in, fitted and copied back on one of three internal
 * streams, so the copies of one chunk overlap the fit of another.  The copies
 * overlap only from pinned host memory (hipHostMalloc); pageable memory
 * works but serialises them.  The pipeline is ordered after the work already
 * queued on `stream`, and `stream` waits for its end; the call returns
 * without waiting, and the host buffers must stay untouched until `stream`
 * reaches that point.  Staging buffers (three chunks) live in the context,
 * sized by p2r_ctx_reserve_host: a call whose chunks or layer count exceed
 * the reservation returns P2R_ENOSPACE without copying or launching
 * anything.  Calls on one context must not overlap.  Not with an MLP. */
/* Sizes the host pipeline's staging (three streams, each one chunk of
 * chunk_tracks tracks, 0 = 131072, rounded up to 256, with max_layers
 * layers, up to 4096) and creates its streams and events.  Grows only;
 * waits for the pipeline's previous work before it reallocates.  The only
 * call that allocates for the pipeline. */
int p2r_ctx_reserve_host(p2r_ctx* ctx, int32_t max_layers, int32_t chunk_tracks);
int p2r_propagate_update_host(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                              const float* layer_r, const float* trk_in, const float* hits, float* trk_out,
                              float* chi2_out, uint32_t* status, int32_t chunk_tracks, void* stream);
int p2z_propagate_update_host(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                              const float* layer_z, const float* trk_in, const float* hits, float* trk_out,
                              float* chi2_out, uint32_t* status, int32_t chunk_tracks, void* stream);

/* Ragged batched fit (paper Section 2's per-track layer loop with per-track
 * layer lists): every track has its own ordered list of surfaces (CSR),
 * each a cylinder (surf_type 0, surf_val = radius) or a plane (surf_type 1,
 * surf_val = signed z), and one 3D hit per surface.
 *   n_tracks tracks, n_hits = offsets[n_tracks] surfaces in total (host
 *   value, used to check sizes; at most P2R_MAX_HITS), max_surfaces >= every
 *   track's count (<= 255; a track with more, or a negative count, is
 *   BAD_INPUT).
 *   offsets [n_tracks+1] (int64, offsets[0] = 0), surf_type [n_hits] (uint8),
 *   surf_val [n_hits], hit_pos [n_hits][3], hit_cov [n_hits][6] (packed; 8-byte aligned),
 *   par_in [n][6], cov_in [n][21], q [n] (int8 +-1); outputs par_out [n][6],
 *   cov_out [n][21], chi2_out [n], status [n].  A surf_type other than 0/1
 *   skips that surface and sets BAD_INPUT.
 * The tracks are counting-sorted on the device by (surface count, |eta|
 * bin); a fit kernel with one wave per block of 64 sorted tracks then
 * streams each block's hits from the CSR arrays through LDS, a few surfaces
 * at a time, the longest blocks first (the autotuner, or p2r_set_variant,
 * picks how many surfaces a chunk holds, the occupancy target, prefetching,
 * and the per-block grid or a persistent grid whose waves take blocks from an
 * atomic counter).  The kernels run as one HIP graph, captured on the first
 * call for a given set of arguments and replayed afterwards (opts->use_graph,
 * non-NULL stream).  The workspace is the one p2r_ctx_reserve sized
 * (P2R_ENOSPACE if it is too small): calls on one context must not overlap.
 * CSR ranges may overlap. */
int fit_tracks_batched(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int64_t n_hits,
                       int32_t max_surfaces, const int64_t* offsets, const uint8_t* surf_type,
                       const float* surf_val, const float* hit_pos, const float* hit_cov,
                       const float* par_in, const float* cov_in, const int8_t* q, float* par_out,
                       float* cov_out, float* chi2_out, uint32_t* status, void* stream);

/* fit_tracks_batched for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, layouts, options and results as
 * fit_tracks_batched, but the sort arrays live in a scratch array that the
 * library holds in static device memory, P2R_NOALLOC_SCRATCH_BYTES on every
 * GPU it runs on (until the process ends), instead of the context's reserved
 * workspace.  Needs no p2r_ctx_reserve; allocates nothing and captures no
 * graph (the kernels are launched directly on `stream`, so the call itself may
 * be captured by the caller).  At most P2R_NOALLOC_MAX_TRACKS tracks
 * (P2R_ENOSPACE beyond, nothing launched).  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * contexts, other threads) race and give wrong results; serialise them. */
int fit_tracks_batched_noalloc(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int64_t n_hits,
                               int32_t max_surfaces, const int64_t* offsets, const uint8_t* surf_type,
                               const float* surf_val, const float* hit_pos, const float* hit_cov,
                               const float* par_in, const float* cov_in, const int8_t* q, float* par_out,
                               float* cov_out, float* chi2_out, uint32_t* status, void* stream);

/* Autotune `which` (0 p2r, 1 p2z, 2 ragged) on synthetic tracks of this
 * shape: times every compiled plain variant with HIP events, keeps the
 * fastest in the context (the default variant unless the fastest beats it by
 * 3% or more) and writes the cache file if the context has one; a shape the
 * cache already holds for this build of the library (its version string names
 * the hash of the sources) is served from it without timing.  p2r / p2z:
 * width, waves per SIMD, layer-loop unroll; n_layers layers.  Ragged:
 * surfaces per staged chunk, waves per SIMD, prefetch, per-block grid or
 * persistent queue, on n_tracks tracks of 5..n_layers mixed cylinders and
 * disks (n_layers = max_surfaces <= 255); it also reserves the ragged
 * workspace for that shape (p2r_ctx_reserve).  Allocates and frees
 * temporary device buffers; synchronises the stream. */
int p2r_autotune(p2r_ctx* ctx, int which, int32_t n_tracks, int32_t n_layers, void* stream);

/* Description of the variant in use for `which` (host string owned by ctx). */
const char* p2r_variant_name(p2r_ctx* ctx, int which);

/* Use the plain variant named `name` (as p2r_variant_name reports it) for
 * `which` (0 p2r, 1 p2z, 2 ragged) from now on, without timing anything:
 * to reproduce a tuned choice, e.g. under a profiler.  P2R_ENOTUNED if no
 * such variant is compiled; the context's choice is then unchanged. */
int p2r_set_variant(p2r_ctx* ctx, int which, const char* name);

/* Name of the i-th compiled plain variant for `which` (0 p2r, 1 p2z,
 * 2 ragged), i = 0, 1, ...; NULL past the last.  Static string. */
const char* p2r_variant_at(int which, int i);

/* ---------------------------------------------------------------------
 * Learned path-length proposal (not in the paper; the north-star
 * extension): an MLP 7 -> 64 -> 64 -> 1 with ReLU, BF16 weights on the
 * matrix cores and FP32 accumulation, that proposes the starting path length
 * of the helix-to-cylinder Newton iteration.  Input: 7 features of the state
 * and the target radius R (p2r_mlp_features); output y with the proposal
 * s0 = s_line (1 + sinh(y) / 100), s_line the straight-line path.  The iteration
 * refines s0, and rejects it (ML_REJECTED, plain start) when |r(s0) - R| >
 * 1e-3 cm.  Parameters: one flat FP32 vector of p2r_mlp_n_params() = 4737
 * values, W1 [64][7], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1]
 * (row-major, y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3).
 * Pass the handle as p2r_opts.mlp to p2r_propagate_update for the learned
 * start.  Buffers are device pointers unless stated. */
typedef struct p2r_mlp p2r_mlp;
/* Allocates the FP32 master weights, Adam state and BF16 copy, and
 * initialises the weights from `seed` (W1, W2 uniform in +-sqrt(6 / fan_in),
 * w3 the same scaled by 0.1, biases 0; a counter-based hash of the seed and
 * the parameter index); synchronises. */
int p2r_mlp_create(p2r_ctx* ctx, p2r_mlp** out, uint64_t seed);
void p2r_mlp_destroy(p2r_mlp* mlp);
int p2r_mlp_n_params(void);
/* host_params: host array of p2r_mlp_n_params() floats; resets Adam; synchronises. */
int p2r_mlp_set_params(p2r_mlp* mlp, const float* host_params);
int p2r_mlp_get_params(p2r_mlp* mlp, float* host_params);
/* Features x [n][7] (and, with s_label [n], targets t [n] = asinh(100 (s_label / s_line - 1));
 * s_line [n] nullable) of states par [n][6], charges q [n] (+-1.0f) and radii R [n]. */
int p2r_mlp_features(p2r_mlp* mlp, const p2r_opts* opts, int32_t n, const float* par, const float* q,
                     const float* R, const float* s_label, float* x, float* t, float* s_line, void* stream);
int p2r_mlp_forward(p2r_mlp* mlp, const float* x, float* y, int32_t B, void* stream);
/* Sizes the per-workgroup gradient partials for batches of up to max_batch
 * (grows only; waits for the device before it reallocates).  The only MLP
 * call besides p2r_mlp_create that allocates. */
int p2r_mlp_reserve(p2r_mlp* mlp, int32_t max_batch);
/* Gradients of the mean squared error over the batch (grads_out [n_params], loss_out [1]; nullable).
 * Deterministic (per-workgroup partials summed in a fixed order).  B must be
 * within p2r_mlp_reserve's max_batch, else P2R_ENOSPACE and nothing runs. */
int p2r_mlp_grads(p2r_mlp* mlp, const float* x, const float* t, int32_t B, float* grads_out,
                  float* loss_out, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the FP32 master weights, then a fresh BF16 copy
 * (same batch limit as p2r_mlp_grads). */
int p2r_mlp_train_step(p2r_mlp* mlp, const float* x, const float* t, int32_t B, float lr,
                       float* loss_out, void* stream);
/* Checkpoint (host file): step, FP32 weights and Adam moments; load restores them bit for bit. */
int p2r_mlp_save(p2r_mlp* mlp, const char* path);
int p2r_mlp_load(p2r_mlp* mlp, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* P2R_H */
