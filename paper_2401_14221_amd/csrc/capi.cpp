// C ABI of libp2r.so: argument checking, variant selection, autotuning and
// the ragged-fit graph.  Declarations and semantics are in include/p2r.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/p2r.h"
#include "launch.h"
#include "mlp.h"
#include "track_math.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(P2R_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Every device allocation of the library goes through here and is counted
// (p2r_device_allocations), so that a test can show that a call made after
// the sizing calls allocates nothing.
std::atomic<unsigned long long> g_allocs{0};
template <typename T>
hipError_t dev_alloc(T** p, size_t bytes) {
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) g_allocs.fetch_add(1, std::memory_order_relaxed);
    return e;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// ------------------------------------------- scratch of the no-alloc fit
// fit_tracks_batched_noalloc works in this array instead of a context's
// workspace: the sort-key histogram and bucket starts (for up to 255
// surfaces per track), the work counter, and the sort arrays (perm, keys,
// run) for up to P2R_NOALLOC_MAX_TRACKS tracks, each at a 256-byte boundary.
// Every GPU the library runs on holds one copy until the process ends.  In
// host code the array's name is not a device address: the address of this
// GPU's copy comes from hipGetSymbolAddress, taken once per device when a
// context is created on it (scratch_setup), and only that address is used.
constexpr size_t NA_KEYS = 256 * p2r::RAG_ETA_BINS + 1;       // sort keys for max_surfaces = 255
constexpr size_t na_round(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t NA_HIST = 0;
constexpr size_t NA_BASE = NA_HIST + na_round(4 * NA_KEYS);
constexpr size_t NA_WORK = NA_BASE + na_round(4 * NA_KEYS);
constexpr size_t NA_PERM = NA_WORK + 256;
constexpr size_t NA_KEYS_OFF = NA_PERM + na_round(4 * (size_t)P2R_NOALLOC_MAX_TRACKS);
constexpr size_t NA_RUN = NA_KEYS_OFF + na_round(4 * (size_t)P2R_NOALLOC_MAX_TRACKS);
constexpr size_t NA_BYTES = NA_RUN + na_round(8 * (size_t)P2R_NOALLOC_MAX_TRACKS);
static_assert(NA_BYTES == P2R_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[NA_MAX_DEVICES] = {};   // this device's copy of `scratch`, or null before setup

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

// Takes this device's address of `scratch` (the device must be current).
int scratch_setup(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return fail(P2R_EINVAL, "device %d beyond %d", device, NA_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return P2R_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (scratch)");
    if (!ptr) return fail(P2R_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = static_cast<char*>(ptr);
    return P2R_OK;
}

char* scratch_of(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

// Arguments a captured ragged graph was recorded with; a call with other
// arguments re-captures.
struct RaggedKey {
    p2r::RaggedLaunch a{};
    p2r::Params P{};
    const void* fn = nullptr;
    hipStream_t stream = nullptr;
    bool same(const RaggedKey& o) const {
        return std::memcmp(&a, &o.a, sizeof a) == 0 && std::memcmp(&P, &o.P, sizeof P) == 0 && fn == o.fn &&
               stream == o.stream;
    }
};

struct p2r_ctx {
    int device = 0;
    std::string arch;
    std::string devname;
    std::string cache_path;
    int cu_count = 0;
    int chosen[3] = {-1, -1, -1};    // variant index per `which`
    std::map<std::string, std::string> cache;  // key -> variant name
    // ragged workspace (owned)
    int32_t* rag_hist = nullptr;
    int32_t* rag_base = nullptr;
    int32_t* rag_work = nullptr;
    int32_t* rag_perm = nullptr;
    int32_t* rag_keys = nullptr;
    int64_t* rag_run = nullptr;
    int32_t rag_n_cap = 0, rag_nkeys_cap = 0, rag_lmax_cap = -1;
    std::vector<int> rag_blocks_per_cu;   // resident workgroups per CU of each ragged fit variant (by index)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    RaggedKey key;
    bool have_graph = false;
    // host pipeline (p2r/p2z_propagate_update_host): streams, events and
    // per-stream staging buffers, created and grown by p2r_ctx_reserve_host
    static constexpr int NPIPE = 3;
    hipStream_t pipe_s[NPIPE] = {};
    hipEvent_t pipe_done[NPIPE] = {};
    hipEvent_t pipe_start = nullptr;
    void* pipe_buf[NPIPE] = {};
    size_t pipe_bytes = 0;
    float* pipe_surf = nullptr;
    int32_t pipe_surf_cap = 0;
};

struct p2r_mlp {
    int device = 0;
    p2r::MlpDev d{};
    void* block = nullptr;   // one allocation holding every buffer
};

namespace {

const p2r::Variant* find_variant(int which, const std::string& name) {
    for (const auto& v : p2r::variants())
        if (v.which == which && name == v.name) return &v;
    return nullptr;
}

int default_variant(int which) {
    const auto& vs = p2r::variants();
    for (size_t i = 0; i < vs.size(); ++i)
        if (vs[i].which == which && !vs[i].learned && !vs[i].fp64 && !vs[i].upd2d) return (int)i;
    return -1;
}

int variant_for(p2r_ctx* ctx, int which, int width, const p2r::Variant** out, bool learned = false,
                bool fp64 = false, bool upd2d = false) {
    const auto& vs = p2r::variants();
    int idx = ctx->chosen[which] >= 0 ? ctx->chosen[which] : default_variant(which);
    if (idx < 0) return fail(P2R_ENOTUNED, "no kernel variant compiled for which=%d", which);
    if (which == 1) upd2d = false;      // planes: the 3D update already is the 2D one
    if (fp64 || upd2d) {
        const int w = width != 0 ? width : vs[idx].width;
        for (const auto& v : vs)
            if (v.which == which && !v.learned && v.fp64 == fp64 && v.upd2d == upd2d && v.width == w) {
                *out = &v;
                return P2R_OK;
            }
        return fail(P2R_ELAYOUT, "no %s%skernel for width %d", fp64 ? "FP64 " : "",
                    upd2d ? "hit-frame-update " : "", w);
    }
    if (learned) {
        const int w = width != 0 ? width : vs[idx].width;
        for (const auto& v : vs)
            if (v.which == which && v.learned && v.width == w) { *out = &v; return P2R_OK; }
        return fail(P2R_ELAYOUT, "no learned-start kernel for width %d", w);
    }
    if (width != 0 && vs[idx].width != width) {
        // first variant of this width (prefer the tuned occupancy/unroll when it matches)
        idx = -1;
        for (size_t i = 0; i < vs.size(); ++i)
            if (vs[i].which == which && vs[i].width == width && !vs[i].learned && !vs[i].fp64 && !vs[i].upd2d) {
                idx = (int)i;
                break;
            }
        if (idx < 0) return fail(P2R_ELAYOUT, "layout width %d not supported (32, 64, 128, 256 for p2r; 64 for p2z)", width);
    }
    (void)0;
    *out = &vs[idx];
    return P2R_OK;
}

p2r::Params params_of(const p2r_opts* o) {
    p2r::Params P;
    P.bz = o->bz_tesla;
    P.tol = o->newton_tol_cm;
    P.max_iter = o->newton_max_iter;
    P.chi2_cut = o->chi2_cut;
    P.fp64_fallback = o->fp64_fallback;
    P.start_mode = o->cyl_start;
    return P;
}

int check_opts(const p2r_opts* o) {
    if (!o) return fail(P2R_EINVAL, "opts is NULL");
    if (!std::isfinite(o->bz_tesla)) return fail(P2R_EINVAL, "bz_tesla not finite");
    if (!(o->newton_tol_cm > 0.0f) || !std::isfinite(o->newton_tol_cm)) return fail(P2R_EINVAL, "newton_tol_cm must be > 0");
    if (o->newton_max_iter < 1 || o->newton_max_iter > 64) return fail(P2R_EINVAL, "newton_max_iter must be in [1, 64]");
    if (std::isnan(o->chi2_cut)) return fail(P2R_EINVAL, "chi2_cut is NaN");
    if (o->fp64_fallback < 0 || o->fp64_fallback > 3) return fail(P2R_EINVAL, "fp64_fallback must be 0, 1, 2 or 3");
    if (o->cyl_start < 0 || o->cyl_start > 1) return fail(P2R_EINVAL, "cyl_start must be 0 or 1");
    if (o->fp64 < 0 || o->fp64 > 1) return fail(P2R_EINVAL, "fp64 must be 0 or 1");
    if (o->update_2d < 0 || o->update_2d > 1) return fail(P2R_EINVAL, "update_2d must be 0 or 1");
    if (o->update_2d && o->mlp) return fail(P2R_EINVAL, "the learned start uses the 3D update (update_2d = 1 with an mlp)");
    if (o->fp64 && o->mlp) return fail(P2R_EINVAL, "the learned start runs in FP32 only (fp64 = 1 with an mlp)");
    return P2R_OK;
}

std::string cache_key(p2r_ctx* ctx, int which, int32_t n, int32_t L) {
    std::ostringstream k;
    k << ctx->arch << "|" << ctx->devname << "|" << which << "|" << n << "|" << L << "|" << p2r_version();
    return k.str();
}

void load_cache(p2r_ctx* ctx) {
    ctx->cache.clear();
    if (ctx->cache_path.empty()) return;
    std::ifstream f(ctx->cache_path);
    if (!f) return;
    // one entry per line: "key" : "variant"   (the file is written by save_cache)
    std::string line;
    while (std::getline(f, line)) {
        size_t a = line.find('"');
        if (a == std::string::npos) continue;
        size_t b = line.find('"', a + 1);
        size_t c = line.find('"', b + 1);
        size_t d = line.find('"', c + 1);
        if (b == std::string::npos || c == std::string::npos || d == std::string::npos) continue;
        ctx->cache[line.substr(a + 1, b - a - 1)] = line.substr(c + 1, d - c - 1);
    }
}

void save_cache(p2r_ctx* ctx) {
    if (ctx->cache_path.empty()) return;
    std::ofstream f(ctx->cache_path, std::ios::trunc);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : ctx->cache)
        f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++i < ctx->cache.size() ? "," : "") << "\n";
    f << "}\n";
}

}  // namespace

namespace p2r {
// synthetic data for the autotuner (kernels.hip)
hipError_t launch_synth(int which, int W, int32_t n, int32_t L, float* surf, float* trk, float* hits, hipStream_t s);
}

extern "C" {

// The version names the hash of the sources the library was built from
// (set by the build); the autotuner's cache keys carry it.
#ifndef P2R_SRC_HASH
#define P2R_SRC_HASH "unhashed"
#endif
const char* p2r_version(void) { return "p2r-mi355x 0.2 src " P2R_SRC_HASH; }

const char* p2r_last_error(void) { return g_err.c_str(); }

void p2r_opts_default(p2r_opts* o) {
    if (!o) return;
    o->bz_tesla = 3.8f;
    o->newton_tol_cm = 1e-6f;
    o->newton_max_iter = 8;
    o->chi2_cut = 0.0f;
    o->fp64_fallback = 3;
    o->width = 0;
    o->mlp = nullptr;
    o->use_graph = 1;
    o->helix_evals = nullptr;
    o->cyl_start = 0;
    o->fp64 = 0;
    o->update_2d = 0;
}

int p2r_ctx_create(p2r_ctx** out, int device, const char* tune_cache_path) {
    if (!out) return fail(P2R_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(P2R_EINVAL, "device %d out of range (%d devices)", device, ndev);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    std::unique_ptr<p2r_ctx> c(new p2r_ctx());
    c->device = device;
    c->arch = prop.gcnArchName;
    c->devname = prop.name;
    c->cu_count = prop.multiProcessorCount;
    if (tune_cache_path) c->cache_path = tune_cache_path;
    load_cache(c.get());
    {
        DeviceGuard g(device);
        if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
        const auto& vs = p2r::variants();
        c->rag_blocks_per_cu.assign(vs.size(), 1);
        for (size_t i = 0; i < vs.size(); ++i) {
            if (vs[i].which != 2) continue;
            int nb = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, vs[i].fn, p2r::RAG_W, 0);
            if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            c->rag_blocks_per_cu[i] = nb > 0 ? nb : 1;
        }
        int rc = scratch_setup(device);
        if (rc) return rc;
    }
    *out = c.release();
    g_err.clear();
    return P2R_OK;
}

void p2r_ctx_destroy(p2r_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    for (int k = 0; k < p2r_ctx::NPIPE; ++k) {
        if (ctx->pipe_s[k]) (void)hipStreamSynchronize(ctx->pipe_s[k]);
        if (ctx->pipe_done[k]) (void)hipEventDestroy(ctx->pipe_done[k]);
        if (ctx->pipe_s[k]) (void)hipStreamDestroy(ctx->pipe_s[k]);
        if (ctx->pipe_buf[k]) (void)hipFree(ctx->pipe_buf[k]);
    }
    if (ctx->pipe_start) (void)hipEventDestroy(ctx->pipe_start);
    if (ctx->pipe_surf) (void)hipFree(ctx->pipe_surf);
    void* bufs[] = {ctx->rag_hist, ctx->rag_base, ctx->rag_work, ctx->rag_perm, ctx->rag_keys, ctx->rag_run};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete ctx;
}

int p2r_layout_width(p2r_ctx* ctx, int which, int32_t* W_out) {
    if (!ctx || !W_out) return fail(P2R_EINVAL, "NULL argument");
    if (which < 0 || which > 2) return fail(P2R_EINVAL, "which must be 0, 1 or 2");
    const p2r::Variant* v = nullptr;
    int rc = variant_for(ctx, which, 0, &v);
    if (rc) return rc;
    *W_out = v->width;
    return P2R_OK;
}

const char* p2r_variant_at(int which, int i) {
    int k = 0;
    for (const auto& v : p2r::variants())
        if (v.which == which && !v.learned && !v.fp64 && !v.upd2d && k++ == i) return v.name;
    return nullptr;
}

int p2r_set_variant(p2r_ctx* ctx, int which, const char* name) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    if (which < 0 || which > 2) return fail(P2R_EINVAL, "which must be 0 (p2r), 1 (p2z) or 2 (ragged)");
    if (!name) return fail(P2R_EINVAL, "name is NULL");
    const p2r::Variant* v = find_variant(which, name);
    if (!v || v->learned || v->fp64 || v->upd2d)
        return fail(P2R_ENOTUNED, "no plain kernel variant named '%s' for which=%d", name, which);
    ctx->chosen[which] = (int)(v - p2r::variants().data());
    return P2R_OK;
}

const char* p2r_variant_name(p2r_ctx* ctx, int which) {
    if (!ctx || which < 0 || which > 2) return "";
    const p2r::Variant* v = nullptr;
    if (variant_for(ctx, which, 0, &v)) return "";
    return v->name;
}

static int propagate_common(int which, p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                            const float* surf, const float* trk_in, const float* hits, float* trk_out,
                            float* chi2_out, uint32_t* status, void* stream) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (n_tracks < 0 || n_layers < 0) return fail(P2R_EINVAL, "negative size (n_tracks %d, n_layers %d)", n_tracks, n_layers);
    if (n_layers > 4096) return fail(P2R_EINVAL, "n_layers %d above 4096", n_layers);
    if (which == 1 && opts->width != 0 && opts->width != 64)
        return fail(P2R_ELAYOUT, "p2z layout width is 64 (got %d)", opts->width);
    if (which == 1 && opts->mlp) return fail(P2R_EINVAL, "the learned start applies to cylinders (p2r) only");
    if (n_tracks == 0) return P2R_OK;
    if (!trk_in || !trk_out || !chi2_out || !status || (n_layers > 0 && (!hits || !surf)))
        return fail(P2R_EINVAL, "NULL buffer");
    const void* ptrs[] = {surf, trk_in, hits, trk_out, chi2_out, status};
    for (const void* p : ptrs)
        if (p && !aligned(p, 4)) return fail(P2R_ELAYOUT, "buffer not 4-byte aligned");
    if ((const void*)trk_in == (const void*)trk_out) return fail(P2R_EINVAL, "trk_in and trk_out must not alias");
    const p2r::Variant* v = nullptr;
    const p2r_mlp* mlp = static_cast<const p2r_mlp*>(opts->mlp);
    if (mlp && mlp->device != ctx->device) return fail(P2R_EINVAL, "mlp lives on device %d, context on %d", mlp->device, ctx->device);
    rc = variant_for(ctx, which, which == 0 ? opts->width : 0, &v, mlp != nullptr, opts->fp64 != 0,
                     opts->update_2d != 0);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    p2r::FitLaunch a{n_tracks, n_layers, surf, trk_in, hits, trk_out, chi2_out, status,
                     mlp ? (const void*)mlp->d.w : nullptr, opts->helix_evals};
    hipError_t e = p2r::launch_fit(*v, a, params_of(opts), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return P2R_OK;
}

int p2r_propagate_update(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                         const float* layer_r, const float* trk_in, const float* hits, float* trk_out,
                         float* chi2_out, uint32_t* status, void* stream) {
    return propagate_common(0, ctx, opts, n_tracks, n_layers, layer_r, trk_in, hits, trk_out, chi2_out, status,
                            stream);
}

int p2z_propagate_update(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                         const float* layer_z, const float* trk_in, const float* hits, float* trk_out,
                         float* chi2_out, uint32_t* status, void* stream) {
    return propagate_common(1, ctx, opts, n_tracks, n_layers, layer_z, trk_in, hits, trk_out, chi2_out, status,
                            stream);
}

// staging of one pipeline stream for chunks of `tracks` (a whole number of
// layout blocks) and n_layers layers: tracks in and out [28][tracks], hits
// [n_layers][9][tracks], chi2 and status [tracks]
static size_t pipe_stage_bytes(int64_t tracks, int32_t n_layers) {
    return sizeof(float) * (size_t)tracks * (2 * 28 + (size_t)n_layers * 9 + 2);
}
static constexpr int32_t PIPE_DEFAULT_CHUNK = 131072;

int p2r_ctx_reserve_host(p2r_ctx* ctx, int32_t max_layers, int32_t chunk_tracks) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    if (max_layers < 0 || max_layers > 4096) return fail(P2R_EINVAL, "max_layers %d outside 0..4096", max_layers);
    if (chunk_tracks < 0) return fail(P2R_EINVAL, "chunk_tracks must be >= 0");
    // any layout width (64, 128 or 256) rounds a chunk up to at most this
    const int64_t tracks = ((int64_t)(chunk_tracks > 0 ? chunk_tracks : PIPE_DEFAULT_CHUNK) + 255) / 256 * 256;
    const size_t bytes = pipe_stage_bytes(tracks, max_layers);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e;
    if (!ctx->pipe_start) {
        for (int k = 0; k < p2r_ctx::NPIPE; ++k) {
            if ((e = hipStreamCreateWithFlags(&ctx->pipe_s[k], hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreateWithFlags");
            if ((e = hipEventCreateWithFlags(&ctx->pipe_done[k], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreateWithFlags");
        }
        if ((e = hipEventCreateWithFlags(&ctx->pipe_start, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreateWithFlags");
    }
    if (bytes > ctx->pipe_bytes) {
        for (int k = 0; k < p2r_ctx::NPIPE; ++k) {
            (void)hipStreamSynchronize(ctx->pipe_s[k]);
            if (ctx->pipe_buf[k]) (void)hipFree(ctx->pipe_buf[k]);
            ctx->pipe_buf[k] = nullptr;
        }
        ctx->pipe_bytes = 0;
        for (int k = 0; k < p2r_ctx::NPIPE; ++k)
            if ((e = dev_alloc(&ctx->pipe_buf[k], bytes)) != hipSuccess) return hip_fail(e, "hipMalloc");
        ctx->pipe_bytes = bytes;
    }
    if (max_layers > ctx->pipe_surf_cap) {
        for (int k = 0; k < p2r_ctx::NPIPE; ++k) (void)hipStreamSynchronize(ctx->pipe_s[k]);
        if (ctx->pipe_surf) (void)hipFree(ctx->pipe_surf);
        ctx->pipe_surf = nullptr;
        ctx->pipe_surf_cap = 0;
        if ((e = dev_alloc(&ctx->pipe_surf, sizeof(float) * (max_layers > 0 ? max_layers : 1))) != hipSuccess)
            return hip_fail(e, "hipMalloc");
        ctx->pipe_surf_cap = max_layers;
    }
    return P2R_OK;
}

// Host-to-host fit in chunks on NPIPE streams: chunk c is copied in, fitted
// and copied back on stream c % NPIPE, into that stream's staging buffers,
// so the copies of one chunk overlap the fit of another; stream order makes
// a staging buffer's reuse wait for its previous chunk.  The pipeline starts
// after the work already queued on `stream` and `stream` waits for its end.
static int propagate_host(int which, p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                          const float* surf, const float* trk_in, const float* hits, float* trk_out,
                          float* chi2_out, uint32_t* status, int32_t chunk_tracks, void* stream) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (opts->mlp) return fail(P2R_EINVAL, "the host pipeline runs the plain fit (no mlp)");
    if (n_tracks < 0 || n_layers < 0) return fail(P2R_EINVAL, "negative size (n_tracks %d, n_layers %d)", n_tracks, n_layers);
    if (n_layers > 4096) return fail(P2R_EINVAL, "n_layers %d above 4096", n_layers);
    if (chunk_tracks < 0) return fail(P2R_EINVAL, "chunk_tracks must be >= 0");
    if (which == 1 && opts->width != 0 && opts->width != 64)
        return fail(P2R_ELAYOUT, "p2z layout width is 64 (got %d)", opts->width);
    if (n_tracks == 0) return P2R_OK;
    if (!trk_in || !trk_out || !chi2_out || !status || (n_layers > 0 && (!hits || !surf)))
        return fail(P2R_EINVAL, "NULL buffer");
    const p2r::Variant* v = nullptr;
    rc = variant_for(ctx, which, which == 0 ? opts->width : 0, &v, false, opts->fp64 != 0, opts->update_2d != 0);
    if (rc) return rc;
    const int W = v->width;
    const int64_t nb = ((int64_t)n_tracks + W - 1) / W;
    int64_t cb = ((int64_t)(chunk_tracks > 0 ? chunk_tracks : PIPE_DEFAULT_CHUNK) + W - 1) / W;   // blocks per chunk
    if (cb > nb) cb = nb;
    const size_t trk_f = (size_t)cb * 28 * W, hit_f = (size_t)cb * n_layers * 9 * W, trk_n = (size_t)cb * W;
    const size_t bytes = pipe_stage_bytes(cb * W, n_layers);   // = 4 (2 trk_f + hit_f + 2 trk_n)
    if (!ctx->pipe_start || bytes > ctx->pipe_bytes || n_layers > ctx->pipe_surf_cap)
        return fail(P2R_ENOSPACE, "host pipeline staging for %lld tracks per chunk and %d layers is not reserved "
                    "(p2r_ctx_reserve_host)", (long long)(cb * W), n_layers);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e;
    hipStream_t us = (hipStream_t)stream;
    // the surface table, then the pipeline, after the caller's queued work
    if (n_layers > 0 &&
        (e = hipMemcpyAsync(ctx->pipe_surf, surf, sizeof(float) * n_layers, hipMemcpyHostToDevice, us)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipEventRecord(ctx->pipe_start, us)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int k = 0; k < p2r_ctx::NPIPE; ++k)
        if ((e = hipStreamWaitEvent(ctx->pipe_s[k], ctx->pipe_start, 0)) != hipSuccess)
            return hip_fail(e, "hipStreamWaitEvent");
    const p2r::Params P = params_of(opts);
    const size_t blk_trk = (size_t)28 * W;               // floats per track block
    const size_t blk_hit = (size_t)n_layers * 9 * W;      // floats of hits per block (all layers)
    int64_t chunk = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += cb, ++chunk) {
        const int k = (int)(chunk % p2r_ctx::NPIPE);
        hipStream_t s = ctx->pipe_s[k];
        const int64_t b1 = std::min(nb, b0 + cb);
        const int64_t nbc = b1 - b0;
        const int64_t t0 = b0 * W;
        const int32_t nc = (int32_t)(std::min<int64_t>(n_tracks, b1 * W) - t0);
        float* st_trk = static_cast<float*>(ctx->pipe_buf[k]);
        float* st_out = st_trk + trk_f;
        float* st_hit = st_out + trk_f;
        float* st_chi2 = st_hit + hit_f;
        uint32_t* st_status = reinterpret_cast<uint32_t*>(st_chi2 + trk_n);
        if ((e = hipMemcpyAsync(st_trk, trk_in + b0 * blk_trk, sizeof(float) * nbc * blk_trk, hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync");
        if (n_layers > 0) {
            if (which == 0) {
                e = hipMemcpyAsync(st_hit, hits + b0 * blk_hit, sizeof(float) * nbc * blk_hit, hipMemcpyHostToDevice, s);
            } else {
                // layer-outer hits: one row of nbc blocks per layer
                const size_t row = sizeof(float) * 9 * W;
                e = hipMemcpy2DAsync(st_hit, row * nbc, hits + b0 * 9 * W, row * nb, row * nbc, n_layers,
                                     hipMemcpyHostToDevice, s);
            }
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (hits)");
        }
        p2r::FitLaunch a{nc, n_layers, ctx->pipe_surf, st_trk, st_hit, st_out, st_chi2, st_status, nullptr,
                         opts->helix_evals};
        if ((e = p2r::launch_fit(*v, a, P, s)) != hipSuccess) return hip_fail(e, "kernel launch");
        if ((e = hipMemcpyAsync(trk_out + b0 * blk_trk, st_out, sizeof(float) * nbc * blk_trk, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(chi2_out + t0, st_chi2, sizeof(float) * nc, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(status + t0, st_status, sizeof(uint32_t) * nc, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync (results)");
    }
    for (int k = 0; k < p2r_ctx::NPIPE; ++k) {
        if ((e = hipEventRecord(ctx->pipe_done[k], ctx->pipe_s[k])) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipStreamWaitEvent(us, ctx->pipe_done[k], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    return P2R_OK;
}

int p2r_propagate_update_host(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                              const float* layer_r, const float* trk_in, const float* hits, float* trk_out,
                              float* chi2_out, uint32_t* status, int32_t chunk_tracks, void* stream) {
    return propagate_host(0, ctx, opts, n_tracks, n_layers, layer_r, trk_in, hits, trk_out, chi2_out, status,
                          chunk_tracks, stream);
}

int p2z_propagate_update_host(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int32_t n_layers,
                              const float* layer_z, const float* trk_in, const float* hits, float* trk_out,
                              float* chi2_out, uint32_t* status, int32_t chunk_tracks, void* stream) {
    return propagate_host(1, ctx, opts, n_tracks, n_layers, layer_z, trk_in, hits, trk_out, chi2_out, status,
                          chunk_tracks, stream);
}

// Launch arguments of the ragged fit over the context's reserved workspace.
static int ragged_launch_args(p2r_ctx* ctx, const p2r::Variant& v, int32_t n_tracks, int64_t n_hits,
                              int32_t max_surfaces, const int64_t* offsets, const uint8_t* surf_type,
                              const float* surf_val, const float* hit_pos, const float* hit_cov,
                              const float* par_in, const float* cov_in, const int8_t* q, float* par_out,
                              float* cov_out, float* chi2_out, uint32_t* status, p2r::RaggedLaunch& a) {
    const int bpc = ctx->rag_blocks_per_cu[&v - p2r::variants().data()];
    a = p2r::RaggedLaunch{};
    a.n = n_tracks;
    a.lmax = max_surfaces;
    a.n_hits = n_hits;
    a.offsets = offsets;
    a.stype = surf_type;
    a.sval = surf_val;
    a.hpos = hit_pos;
    a.hcov = hit_cov;
    a.par_in = par_in;
    a.cov_in = cov_in;
    a.q = q;
    a.par_out = par_out;
    a.cov_out = cov_out;
    a.chi2 = chi2_out;
    a.status = status;
    a.hist = ctx->rag_hist;
    a.base = ctx->rag_base;
    a.work = ctx->rag_work;
    a.perm = ctx->rag_perm;
    a.keys = ctx->rag_keys;
    a.run = ctx->rag_run;
    a.nkeys = p2r::ragged_nkeys(max_surfaces);
    a.nb = (n_tracks + p2r::RAG_W - 1) / p2r::RAG_W;
    a.grid = std::min(a.nb, ctx->cu_count * bpc);
    return P2R_OK;
}

int p2r_ctx_reserve(p2r_ctx* ctx, int32_t max_tracks, int32_t max_surfaces) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    if (max_tracks < 0) return fail(P2R_EINVAL, "negative max_tracks");
    if (max_surfaces < 0 || max_surfaces > 255) return fail(P2R_EINVAL, "max_surfaces must be in [0, 255]");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e;
    const int nkeys = p2r::ragged_nkeys(max_surfaces);
    const bool grow_n = max_tracks > ctx->rag_n_cap, grow_k = nkeys > ctx->rag_nkeys_cap;
    if (grow_n || grow_k) {
        // a captured graph records the old buffers
        if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->exec = nullptr;
        ctx->graph = nullptr;
        ctx->have_graph = false;
    }
    if (grow_n) {
        for (int32_t** b : {&ctx->rag_perm, &ctx->rag_keys}) {
            if (*b) (void)hipFree(*b);
            *b = nullptr;
        }
        if (ctx->rag_run) (void)hipFree(ctx->rag_run);
        ctx->rag_run = nullptr;
        ctx->rag_n_cap = 0;
        const size_t n = (size_t)std::max(max_tracks, 1);
        if ((e = dev_alloc(&ctx->rag_perm, sizeof(int32_t) * n)) != hipSuccess ||
            (e = dev_alloc(&ctx->rag_keys, sizeof(int32_t) * n)) != hipSuccess ||
            (e = dev_alloc(&ctx->rag_run, sizeof(int64_t) * n)) != hipSuccess)
            return hip_fail(e, "hipMalloc (ragged workspace)");
        ctx->rag_n_cap = max_tracks;
    }
    if (grow_k) {
        for (int32_t** b : {&ctx->rag_hist, &ctx->rag_base}) {
            if (*b) (void)hipFree(*b);
            *b = nullptr;
        }
        ctx->rag_nkeys_cap = 0;
        if ((e = dev_alloc(&ctx->rag_hist, sizeof(int32_t) * nkeys)) != hipSuccess ||
            (e = dev_alloc(&ctx->rag_base, sizeof(int32_t) * nkeys)) != hipSuccess)
            return hip_fail(e, "hipMalloc (ragged workspace)");
        ctx->rag_nkeys_cap = nkeys;
    }
    ctx->rag_lmax_cap = std::max(ctx->rag_lmax_cap, max_surfaces);
    if (!ctx->rag_work && (e = dev_alloc(&ctx->rag_work, sizeof(int32_t))) != hipSuccess)
        return hip_fail(e, "hipMalloc (ragged workspace)");
    return P2R_OK;
}

unsigned long long p2r_device_allocations(void) { return g_allocs.load(std::memory_order_relaxed); }

// Argument checks shared by the ragged entry points (nothing launched on
// failure); *v gets the variant the context uses.  Returns 1 (no error,
// nothing to do) for an empty problem.
static int ragged_check(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int64_t n_hits, int32_t max_surfaces,
                        const int64_t* offsets, const uint8_t* surf_type, const float* surf_val,
                        const float* hit_pos, const float* hit_cov, const float* par_in, const float* cov_in,
                        const int8_t* q, float* par_out, float* cov_out, float* chi2_out, uint32_t* status,
                        const p2r::Variant** v) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (opts->mlp) return fail(P2R_EINVAL, "the learned start is not available in the ragged fit");
    if (n_tracks < 0 || n_hits < 0) return fail(P2R_EINVAL, "negative size (n_tracks %d, n_hits %lld)", n_tracks,
                                                (long long)n_hits);
    if (max_surfaces < 0 || max_surfaces > 255) return fail(P2R_EINVAL, "max_surfaces must be in [0, 255]");
    if (n_hits > (int64_t)n_tracks * max_surfaces)
        return fail(P2R_EINVAL, "n_hits %lld exceeds n_tracks * max_surfaces", (long long)n_hits);
    // the fit addresses the CSR arrays with 32-bit byte offsets (hit_cov, 24 B per surface, the largest)
    if (n_hits > P2R_MAX_HITS)
        return fail(P2R_EINVAL, "n_hits %lld too large for one call (at most %lld)", (long long)n_hits,
                    (long long)P2R_MAX_HITS);
    if (n_tracks == 0) return 1;
    if (!offsets || !par_in || !cov_in || !q || !par_out || !cov_out || !chi2_out || !status ||
        (n_hits > 0 && (!surf_type || !surf_val || !hit_pos || !hit_cov)))
        return fail(P2R_EINVAL, "NULL buffer");
    const void* a4[] = {surf_val, hit_pos, hit_cov, par_in, cov_in, par_out, cov_out, chi2_out, status};
    if (!aligned(offsets, 8)) return fail(P2R_ELAYOUT, "offsets not 8-byte aligned");
    if (hit_cov && !aligned(hit_cov, 8)) return fail(P2R_ELAYOUT, "hit_cov not 8-byte aligned");
    for (const void* p : a4)
        if (p && !aligned(p, 4)) return fail(P2R_ELAYOUT, "buffer not 4-byte aligned");
    return variant_for(ctx, 2, 0, v, false, opts->fp64 != 0, opts->update_2d != 0);
}

int fit_tracks_batched(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int64_t n_hits, int32_t max_surfaces,
                       const int64_t* offsets, const uint8_t* surf_type, const float* surf_val,
                       const float* hit_pos, const float* hit_cov, const float* par_in, const float* cov_in,
                       const int8_t* q, float* par_out, float* cov_out, float* chi2_out, uint32_t* status,
                       void* stream) {
    const p2r::Variant* v = nullptr;
    int rc = ragged_check(ctx, opts, n_tracks, n_hits, max_surfaces, offsets, surf_type, surf_val, hit_pos, hit_cov,
                          par_in, cov_in, q, par_out, cov_out, chi2_out, status, &v);
    if (rc) return rc > 0 ? P2R_OK : rc;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    // the workspace comes from p2r_ctx_reserve: nothing is allocated here
    const int nkeys = p2r::ragged_nkeys(max_surfaces);
    if (n_tracks > ctx->rag_n_cap || nkeys > ctx->rag_nkeys_cap || !ctx->rag_work)
        return fail(P2R_ENOSPACE, "ragged workspace reserved for %d tracks and %d surfaces per track; this call "
                    "needs %d and %d: call p2r_ctx_reserve first", ctx->rag_n_cap, ctx->rag_lmax_cap, n_tracks,
                    max_surfaces);
    hipError_t e;
    p2r::RaggedLaunch a{};
    if ((rc = ragged_launch_args(ctx, *v, n_tracks, n_hits, max_surfaces, offsets, surf_type, surf_val, hit_pos,
                                 hit_cov, par_in, cov_in, q, par_out, cov_out, chi2_out, status, a)))
        return rc;
    p2r::Params P = params_of(opts);
    hipStream_t s = (hipStream_t)stream;
    if (!opts->use_graph || s == nullptr) {
        e = p2r::launch_ragged(*v, a, P, s);
        if (e != hipSuccess) return hip_fail(e, "ragged launch");
        return P2R_OK;
    }
    RaggedKey k;
    k.a = a;
    k.P = P;
    k.fn = v->fn;
    k.stream = s;
    if (!ctx->have_graph || !ctx->key.same(k)) {
        if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->exec = nullptr;
        ctx->graph = nullptr;
        ctx->have_graph = false;
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        hipError_t el = p2r::launch_ragged(*v, a, P, s);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (el != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(el, "ragged launch during capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        ctx->graph = graph;
        ctx->exec = exec;
        ctx->key = k;
        ctx->have_graph = true;
    }
    if ((e = hipGraphLaunch(ctx->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return P2R_OK;
}

int fit_tracks_batched_noalloc(p2r_ctx* ctx, const p2r_opts* opts, int32_t n_tracks, int64_t n_hits,
                               int32_t max_surfaces, const int64_t* offsets, const uint8_t* surf_type,
                               const float* surf_val, const float* hit_pos, const float* hit_cov,
                               const float* par_in, const float* cov_in, const int8_t* q, float* par_out,
                               float* cov_out, float* chi2_out, uint32_t* status, void* stream) {
    const p2r::Variant* v = nullptr;
    int rc = ragged_check(ctx, opts, n_tracks, n_hits, max_surfaces, offsets, surf_type, surf_val, hit_pos, hit_cov,
                          par_in, cov_in, q, par_out, cov_out, chi2_out, status, &v);
    if (rc) return rc > 0 ? P2R_OK : rc;
    if (n_tracks > P2R_NOALLOC_MAX_TRACKS)
        return fail(P2R_ENOSPACE, "fit_tracks_batched_noalloc takes at most %d tracks (got %d)",
                    (int)P2R_NOALLOC_MAX_TRACKS, n_tracks);
    char* base = scratch_of(ctx->device);
    if (!base) return fail(P2R_EHIP, "no scratch address for device %d", ctx->device);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    p2r::RaggedLaunch a{};
    if ((rc = ragged_launch_args(ctx, *v, n_tracks, n_hits, max_surfaces, offsets, surf_type, surf_val, hit_pos,
                                 hit_cov, par_in, cov_in, q, par_out, cov_out, chi2_out, status, a)))
        return rc;
    // the sort arrays in this GPU's scratch instead of the context's workspace;
    // rag_reset (a kernel) clears the histogram and the work counter each call
    a.hist = reinterpret_cast<int32_t*>(base + NA_HIST);
    a.base = reinterpret_cast<int32_t*>(base + NA_BASE);
    a.work = reinterpret_cast<int32_t*>(base + NA_WORK);
    a.perm = reinterpret_cast<int32_t*>(base + NA_PERM);
    a.keys = reinterpret_cast<int32_t*>(base + NA_KEYS_OFF);
    a.run = reinterpret_cast<int64_t*>(base + NA_RUN);
    const hipError_t e = p2r::launch_ragged(*v, a, params_of(opts), (hipStream_t)stream);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "ragged launch");
}

// ------------------------------------------------------------------- MLP

static int mlp_check(p2r_mlp* m) { return m ? P2R_OK : fail(P2R_EINVAL, "mlp is NULL"); }

// Initial weights from a seed: W1, W2 uniform in +-sqrt(6 / fan_in), w3 the
// same times 0.1, biases 0; element k of the flat vector draws
// hash_u01(seed-derived key, k).
static void mlp_init_params(uint64_t seed, std::vector<float>& w) {
    w.assign(p2r::MLP_NPARAM, 0.0f);
    const uint32_t key = (uint32_t)(seed ^ (seed >> 32)) * 0x9E3779B1u + 0x6D4C5031u;
    const int nin = 7, nh = 64;
    auto fill = [&](size_t off, size_t count, int fan_in, float scale) {
        const float lim = std::sqrt(6.0f / (float)fan_in) * scale;
        for (size_t k = 0; k < count; ++k)
            w[off + k] = (2.0f * p2r::hash_u01(key, (uint32_t)(off + k)) - 1.0f) * lim;
    };
    size_t o = 0;
    fill(o, (size_t)nh * nin, nin, 1.0f);  o += (size_t)nh * nin + nh;        // W1, b1 = 0
    fill(o, (size_t)nh * nh, nh, 1.0f);    o += (size_t)nh * nh + nh;         // W2, b2 = 0
    fill(o, (size_t)nh, nh, 0.1f);                                            // w3, b3 = 0
}

int p2r_mlp_create(p2r_ctx* ctx, p2r_mlp** out, uint64_t seed) {
    if (!ctx || !out) return fail(P2R_EINVAL, "NULL argument");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    std::unique_ptr<p2r_mlp> m(new p2r_mlp());
    m->device = ctx->device;
    const size_t np = p2r::MLP_NPARAM;
    const size_t fl = (4 * np + 64) * sizeof(float);
    const size_t bytes = fl + sizeof(p2r::MlpWeights) + 256;
    hipError_t e = dev_alloc(&m->block, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMemset(m->block, 0, bytes)) != hipSuccess) { (void)hipFree(m->block); return hip_fail(e, "hipMemset"); }
    float* f = static_cast<float*>(m->block);
    m->d.master = f;
    m->d.m = f + np;
    m->d.v = f + 2 * np;
    m->d.grad = f + 3 * np;
    m->d.loss = f + 4 * np;
    uintptr_t wp = (reinterpret_cast<uintptr_t>(f + 4 * np + 64) + 255) & ~uintptr_t(255);
    m->d.w = reinterpret_cast<p2r::MlpWeights*>(wp);
    m->d.step = 0;
    std::vector<float> w;
    mlp_init_params(seed, w);
    if ((e = hipMemcpy(m->d.master, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = p2r::mlp_recast(m->d, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        (void)hipFree(m->block);
        return hip_fail(e, "p2r_mlp_create (initial weights)");
    }
    *out = m.release();
    return P2R_OK;
}

void p2r_mlp_destroy(p2r_mlp* m) {
    if (!m) return;
    DeviceGuard g(m->device);
    if (m->block) (void)hipFree(m->block);
    if (m->d.part) (void)hipFree(m->d.part);
    delete m;
}

// per-workgroup gradient rows for batches up to B
int p2r_mlp_reserve(p2r_mlp* m, int32_t B) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (B <= 0) return fail(P2R_EINVAL, "batch must be positive");
    const int nb = p2r::mlp_grad_blocks(B);
    if (nb <= m->d.part_blocks) return P2R_OK;
    DeviceGuard g(m->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    (void)hipDeviceSynchronize();          // earlier gradient calls may still read the old rows
    if (m->d.part) (void)hipFree(m->d.part);
    m->d.part = nullptr;
    m->d.part_blocks = 0;
    hipError_t e = dev_alloc(&m->d.part, (size_t)nb * (p2r::MLP_NPARAM + 1) * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    m->d.part_blocks = nb;
    return P2R_OK;
}

int p2r_mlp_set_params(p2r_mlp* m, const float* host_params) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!host_params) return fail(P2R_EINVAL, "host_params is NULL");
    DeviceGuard g(m->device);
    const size_t nb = p2r::MLP_NPARAM * sizeof(float);
    hipError_t e = hipMemcpy(m->d.master, host_params, nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->d.m, 0, 2 * nb);
    if (e == hipSuccess) e = p2r::mlp_recast(m->d, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "p2r_mlp_set_params");
    m->d.step = 0;
    return P2R_OK;
}

int p2r_mlp_get_params(p2r_mlp* m, float* host_params) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!host_params) return fail(P2R_EINVAL, "host_params is NULL");
    DeviceGuard g(m->device);
    hipError_t e = hipMemcpy(host_params, m->d.master, p2r::MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "p2r_mlp_get_params");
}

int p2r_mlp_n_params(void) { return p2r::MLP_NPARAM; }

int p2r_mlp_features(p2r_mlp* m, const p2r_opts* opts, int32_t n, const float* par, const float* q, const float* R,
                     const float* s_label, float* x, float* t, float* s_line, void* stream) {
    int rc = mlp_check(m);
    if (!rc) rc = check_opts(opts);
    if (rc) return rc;
    if (n < 0) return fail(P2R_EINVAL, "negative n");
    if (n == 0) return P2R_OK;
    if (!par || !q || !R || !x || (t && !s_label)) return fail(P2R_EINVAL, "NULL buffer");
    DeviceGuard g(m->device);
    hipError_t e = p2r::mlp_features(n, par, q, R, s_label, opts->bz_tesla, x, t, s_line, (hipStream_t)stream);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "mlp features");
}

int p2r_mlp_forward(p2r_mlp* m, const float* x, float* y, int32_t B, void* stream) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (B < 0) return fail(P2R_EINVAL, "negative batch");
    if (B > 0 && (!x || !y)) return fail(P2R_EINVAL, "NULL buffer");
    DeviceGuard g(m->device);
    hipError_t e = p2r::mlp_forward(m->d, x, y, B, (hipStream_t)stream);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "mlp forward");
}

int p2r_mlp_grads(p2r_mlp* m, const float* x, const float* t, int32_t B, float* grads_out, float* loss_out,
                  void* stream) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (B <= 0) return fail(P2R_EINVAL, "batch must be positive");
    if (!x || !t) return fail(P2R_EINVAL, "NULL buffer");
    if (p2r::mlp_grad_blocks(B) > m->d.part_blocks)
        return fail(P2R_ENOSPACE, "gradient partials for a batch of %d are not reserved (p2r_mlp_reserve)", B);
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = p2r::mlp_grads(m->d, x, t, B, s);
    if (e == hipSuccess && grads_out)
        e = hipMemcpyAsync(grads_out, m->d.grad, p2r::MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && loss_out) e = hipMemcpyAsync(loss_out, m->d.loss, sizeof(float), hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "mlp grads");
}

int p2r_mlp_train_step(p2r_mlp* m, const float* x, const float* t, int32_t B, float lr, float* loss_out,
                       void* stream) {
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(P2R_EINVAL, "lr must be > 0");
    int rc = p2r_mlp_grads(m, x, t, B, nullptr, loss_out, stream);
    if (rc) return rc;
    DeviceGuard g(m->device);
    m->d.step += 1;
    hipError_t e = p2r::mlp_adam(m->d, lr, m->d.step, (hipStream_t)stream);
    return e == hipSuccess ? P2R_OK : hip_fail(e, "mlp adam");
}

// checkpoint: magic, step, then master weights, Adam m and v (FP32)
int p2r_mlp_save(p2r_mlp* m, const char* path) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!path) return fail(P2R_EINVAL, "path is NULL");
    DeviceGuard g(m->device);
    std::vector<float> buf(3 * (size_t)p2r::MLP_NPARAM);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(buf.data(), m->d.master, buf.size() * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "p2r_mlp_save");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(P2R_EINVAL, "cannot open %s", path);
    const uint32_t hdr[4] = {0x504D4C50u /* "PLMP" */, 1u, (uint32_t)p2r::MLP_NPARAM, (uint32_t)m->d.step};
    bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? P2R_OK : fail(P2R_EINVAL, "write to %s failed", path);
}

int p2r_mlp_load(p2r_mlp* m, const char* path) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!path) return fail(P2R_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(P2R_EINVAL, "cannot open %s", path);
    uint32_t hdr[4];
    std::vector<float> buf(3 * (size_t)p2r::MLP_NPARAM);
    bool ok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x504D4C50u && hdr[1] == 1u &&
              hdr[2] == (uint32_t)p2r::MLP_NPARAM && std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(P2R_EINVAL, "%s is not a p2r MLP checkpoint", path);
    DeviceGuard g(m->device);
    hipError_t e = hipMemcpy(m->d.master, buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = p2r::mlp_recast(m->d, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "p2r_mlp_load");
    m->d.step = (int32_t)hdr[3];
    return P2R_OK;
}


// Ragged autotune: every plain ragged variant (chunk of staged surfaces,
// waves per SIMD, per-block grid or persistent queue, prefetch) timed on
// synthetic tracks with n surfaces each drawn from 5 .. lmax, mixed
// cylinders and disks in crossing order.  Reserves the context's ragged
// workspace for this shape.
static int autotune_ragged(p2r_ctx* ctx, const std::string& key, int32_t n, int32_t lmax, hipStream_t s) {
    const auto& vs = p2r::variants();
    std::vector<int64_t> off((size_t)n + 1, 0);
    for (int32_t t = 0; t < n; ++t) off[t + 1] = off[t] + p2r::ragged_synth_count(t, lmax);
    const int64_t H = off[n];
    if (H > P2R_MAX_HITS) return fail(P2R_EINVAL, "ragged autotune: too many surfaces");
    int rc = p2r_ctx_reserve(ctx, n, lmax);
    if (rc) return rc;
    int64_t* d_off = nullptr;
    uint8_t* d_st = nullptr;
    float *d_sv = nullptr, *d_hp = nullptr, *d_hc = nullptr, *d_par = nullptr, *d_cov = nullptr;
    float *d_po = nullptr, *d_co = nullptr, *d_c2 = nullptr;
    int8_t* d_q = nullptr;
    uint32_t* d_status = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (void* p : {(void*)d_off, (void*)d_st, (void*)d_sv, (void*)d_hp, (void*)d_hc, (void*)d_par, (void*)d_cov,
                        (void*)d_po, (void*)d_co, (void*)d_c2, (void*)d_q, (void*)d_status})
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
#define TRY(x, what)                              \
    do {                                          \
        e = (x);                                  \
        if (e != hipSuccess) {                    \
            cleanup();                            \
            return hip_fail(e, what);             \
        }                                         \
    } while (0)
    const size_t h1 = (size_t)std::max<int64_t>(H, 1);
    TRY(dev_alloc(&d_off, sizeof(int64_t) * (n + 1)), "hipMalloc");
    TRY(dev_alloc(&d_st, h1), "hipMalloc");
    TRY(dev_alloc(&d_sv, sizeof(float) * h1), "hipMalloc");
    TRY(dev_alloc(&d_hp, sizeof(float) * 3 * h1), "hipMalloc");
    TRY(dev_alloc(&d_hc, sizeof(float) * 6 * h1), "hipMalloc");
    TRY(dev_alloc(&d_par, sizeof(float) * 6 * n), "hipMalloc");
    TRY(dev_alloc(&d_cov, sizeof(float) * 21 * n), "hipMalloc");
    TRY(dev_alloc(&d_po, sizeof(float) * 6 * n), "hipMalloc");
    TRY(dev_alloc(&d_co, sizeof(float) * 21 * n), "hipMalloc");
    TRY(dev_alloc(&d_c2, sizeof(float) * n), "hipMalloc");
    TRY(dev_alloc(&d_q, (size_t)n), "hipMalloc");
    TRY(dev_alloc(&d_status, sizeof(uint32_t) * n), "hipMalloc");
    TRY(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    TRY(p2r::launch_ragged_synth(n, lmax, d_off, d_st, d_sv, d_hp, d_hc, d_par, d_cov, d_q, s), "synthetic fill");
    TRY(hipEventCreate(&e0), "hipEventCreate");
    TRY(hipEventCreate(&e1), "hipEventCreate");
    p2r_opts o;
    p2r_opts_default(&o);
    o.chi2_cut = 30.0f;
    const p2r::Params P = params_of(&o);
    const int def = default_variant(2);
    float best = 1e30f, def_ms = -1.0f;
    int best_i = -1;
    for (size_t i = 0; i < vs.size(); ++i) {
        if (vs[i].which != 2 || vs[i].learned || vs[i].fp64 || vs[i].upd2d) continue;
        p2r::RaggedLaunch a{};
        if ((rc = ragged_launch_args(ctx, vs[i], n, H, lmax, d_off, d_st, d_sv, d_hp, d_hc, d_par, d_cov, d_q, d_po,
                                     d_co, d_c2, d_status, a))) {
            cleanup();
            return rc;
        }
        for (int w = 0; w < 2; ++w) TRY(p2r::launch_ragged(vs[i], a, P, s), "ragged launch");
        TRY(hipEventRecord(e0, s), "hipEventRecord");
        const int reps = 5;
        for (int r = 0; r < reps; ++r) TRY(p2r::launch_ragged(vs[i], a, P, s), "ragged launch");
        TRY(hipEventRecord(e1, s), "hipEventRecord");
        TRY(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (ms < best) { best = ms; best_i = (int)i; }
        if ((int)i == def) def_ms = ms;
    }
    cleanup();
#undef TRY
    if (best_i < 0) return fail(P2R_ENOTUNED, "no ragged variant");
    if (def_ms > 0.0f && best >= 0.97f * def_ms) best_i = def;
    ctx->chosen[2] = best_i;
    ctx->cache[key] = vs[best_i].name;
    save_cache(ctx);
    return P2R_OK;
}

int p2r_autotune(p2r_ctx* ctx, int which, int32_t n_tracks, int32_t n_layers, void* stream) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    if (which < 0 || which > 2) return fail(P2R_EINVAL, "autotune supports which = 0 (p2r), 1 (p2z) or 2 (ragged)");
    if (n_tracks <= 0 || n_layers <= 0) return fail(P2R_EINVAL, "autotune needs n_tracks > 0 and n_layers > 0");
    if (which == 2 && n_layers > 255) return fail(P2R_EINVAL, "ragged autotune: max_surfaces must be in [1, 255]");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const auto& vs = p2r::variants();
    std::string key = cache_key(ctx, which, n_tracks, n_layers);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) {
        if (const p2r::Variant* v = find_variant(which, it->second)) {
            ctx->chosen[which] = (int)(v - vs.data());
            return which == 2 ? p2r_ctx_reserve(ctx, n_tracks, n_layers) : P2R_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (which == 2) return autotune_ragged(ctx, key, n_tracks, n_layers, s);
    const size_t nb256 = ((size_t)n_tracks + 255) / 256;
    const size_t trk_sz = nb256 * 256 * 28, hit_sz = nb256 * 256 * 9 * (size_t)n_layers;
    float *surf = nullptr, *trk = nullptr, *hits = nullptr, *out = nullptr, *chi2 = nullptr;
    uint32_t* st = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (void* p : {(void*)surf, (void*)trk, (void*)hits, (void*)out, (void*)chi2, (void*)st})
            if (p) (void)hipFree(p);
    };
#define TRY(x, what)                              \
    do {                                          \
        e = (x);                                  \
        if (e != hipSuccess) {                    \
            cleanup();                            \
            return hip_fail(e, what);             \
        }                                         \
    } while (0)
    TRY(dev_alloc(&surf, sizeof(float) * n_layers), "hipMalloc");
    TRY(dev_alloc(&trk, sizeof(float) * trk_sz), "hipMalloc");
    TRY(dev_alloc(&hits, sizeof(float) * hit_sz), "hipMalloc");
    TRY(dev_alloc(&out, sizeof(float) * trk_sz), "hipMalloc");
    TRY(dev_alloc(&chi2, sizeof(float) * n_tracks), "hipMalloc");
    TRY(dev_alloc(&st, sizeof(uint32_t) * n_tracks), "hipMalloc");
    hipEvent_t e0, e1;
    TRY(hipEventCreate(&e0), "hipEventCreate");
    TRY(hipEventCreate(&e1), "hipEventCreate");
    p2r_opts o;
    p2r_opts_default(&o);
    p2r::Params P = params_of(&o);
    float best = 1e30f, def_ms = -1.f;
    int best_i = -1;
    int cur_w = -1;
    for (size_t i = 0; i < vs.size(); ++i) {
        if (vs[i].which != which || vs[i].learned || vs[i].fp64 || vs[i].upd2d) continue;
        if (vs[i].width != cur_w) {
            TRY(p2r::launch_synth(which, vs[i].width, n_tracks, n_layers, surf, trk, hits, s), "synthetic fill");
            cur_w = vs[i].width;
        }
        p2r::FitLaunch a{n_tracks, n_layers, surf, trk, hits, out, chi2, st, nullptr, nullptr};
        for (int w = 0; w < 2; ++w) TRY(p2r::launch_fit(vs[i], a, P, s), "kernel launch");
        TRY(hipEventRecord(e0, s), "hipEventRecord");
        const int reps = 5;
        for (int r = 0; r < reps; ++r) TRY(p2r::launch_fit(vs[i], a, P, s), "kernel launch");
        TRY(hipEventRecord(e1, s), "hipEventRecord");
        TRY(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (ms < best) { best = ms; best_i = (int)i; }
        if ((int)i == default_variant(which)) def_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
#undef TRY
    if (best_i < 0) return fail(P2R_ENOTUNED, "no variant for which=%d", which);
    // keep the default unless another variant is clearly faster: variants
    // within a few percent trade places from run to run
    if (def_ms > 0.f && best >= 0.97f * def_ms) best_i = default_variant(which);
    ctx->chosen[which] = best_i;
    ctx->cache[key] = vs[best_i].name;
    save_cache(ctx);
    return P2R_OK;
}

}  // extern "C"
