// C ABI of libp2r.so: argument checking, variant selection, autotuning and
// the ragged-fit graph.  Declarations and semantics are in include/p2r.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/p2r.h"
#include "launch.h"
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

}  // namespace

struct RaggedShape {
    int32_t n = -1;
    int64_t H = -1;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t stream = nullptr;
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
    p2r::RaggedLaunch rag{};
    size_t rag_n_cap = 0, rag_nb_cap = 0;
    int rag_lmax = 0;
    RaggedShape shape;
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
        if (vs[i].which == which) return (int)i;
    return -1;
}

int variant_for(p2r_ctx* ctx, int which, int width, const p2r::Variant** out) {
    const auto& vs = p2r::variants();
    int idx = ctx->chosen[which] >= 0 ? ctx->chosen[which] : default_variant(which);
    if (idx < 0) return fail(P2R_ENOTUNED, "no kernel variant compiled for which=%d", which);
    if (width != 0 && vs[idx].width != width) {
        // first variant of this width (prefer the tuned occupancy/unroll when it matches)
        idx = -1;
        for (size_t i = 0; i < vs.size(); ++i)
            if (vs[i].which == which && vs[i].width == width) { idx = (int)i; break; }
        if (idx < 0) return fail(P2R_ELAYOUT, "layout width %d not supported (32, 64, 128, 256 for p2r; 64 for p2z)", width);
    }
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
    return P;
}

int check_opts(const p2r_opts* o) {
    if (!o) return fail(P2R_EINVAL, "opts is NULL");
    if (!std::isfinite(o->bz_tesla)) return fail(P2R_EINVAL, "bz_tesla not finite");
    if (!(o->newton_tol_cm > 0.0f) || !std::isfinite(o->newton_tol_cm)) return fail(P2R_EINVAL, "newton_tol_cm must be > 0");
    if (o->newton_max_iter < 1 || o->newton_max_iter > 64) return fail(P2R_EINVAL, "newton_max_iter must be in [1, 64]");
    if (std::isnan(o->chi2_cut)) return fail(P2R_EINVAL, "chi2_cut is NaN");
    if (o->fp64_fallback < 0 || o->fp64_fallback > 2) return fail(P2R_EINVAL, "fp64_fallback must be 0, 1 or 2");
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

const char* p2r_version(void) { return "p2r-mi355x 0.1"; }

const char* p2r_last_error(void) { return g_err.c_str(); }

void p2r_opts_default(p2r_opts* o) {
    if (!o) return;
    o->bz_tesla = 3.8f;
    o->newton_tol_cm = 1e-6f;
    o->newton_max_iter = 8;
    o->chi2_cut = 0.0f;
    o->fp64_fallback = 1;
    o->width = 0;
    o->mlp = nullptr;
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
    *out = c.release();
    g_err.clear();
    return P2R_OK;
}

void p2r_ctx_destroy(p2r_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (ctx->shape.exec) (void)hipGraphExecDestroy(ctx->shape.exec);
    if (ctx->shape.graph) (void)hipGraphDestroy(ctx->shape.graph);
    void* bufs[] = {ctx->rag.counts, ctx->rag.perm, ctx->rag.work, ctx->rag.trk_pack, ctx->rag.hit_pack,
                    ctx->rag.blk_len};
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
    rc = variant_for(ctx, which, which == 0 ? opts->width : 0, &v);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    p2r::FitLaunch a{n_tracks, n_layers, surf, trk_in, hits, trk_out, chi2_out, status, opts->mlp};
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

int p2r_autotune(p2r_ctx* ctx, int which, int32_t n_tracks, int32_t n_layers, void* stream) {
    if (!ctx) return fail(P2R_EINVAL, "ctx is NULL");
    if (which < 0 || which > 1) return fail(P2R_EINVAL, "autotune supports which = 0 (p2r) or 1 (p2z)");
    if (n_tracks <= 0 || n_layers <= 0) return fail(P2R_EINVAL, "autotune needs n_tracks > 0 and n_layers > 0");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const auto& vs = p2r::variants();
    std::string key = cache_key(ctx, which, n_tracks, n_layers);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) {
        if (const p2r::Variant* v = find_variant(which, it->second)) {
            ctx->chosen[which] = (int)(v - vs.data());
            return P2R_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
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
    TRY(hipMalloc(&surf, sizeof(float) * n_layers), "hipMalloc");
    TRY(hipMalloc(&trk, sizeof(float) * trk_sz), "hipMalloc");
    TRY(hipMalloc(&hits, sizeof(float) * hit_sz), "hipMalloc");
    TRY(hipMalloc(&out, sizeof(float) * trk_sz), "hipMalloc");
    TRY(hipMalloc(&chi2, sizeof(float) * n_tracks), "hipMalloc");
    TRY(hipMalloc(&st, sizeof(uint32_t) * n_tracks), "hipMalloc");
    hipEvent_t e0, e1;
    TRY(hipEventCreate(&e0), "hipEventCreate");
    TRY(hipEventCreate(&e1), "hipEventCreate");
    p2r_opts o;
    p2r_opts_default(&o);
    p2r::Params P = params_of(&o);
    float best = 1e30f;
    int best_i = -1;
    int cur_w = -1;
    for (size_t i = 0; i < vs.size(); ++i) {
        if (vs[i].which != which) continue;
        if (vs[i].width != cur_w) {
            TRY(p2r::launch_synth(which, vs[i].width, n_tracks, n_layers, surf, trk, hits, s), "synthetic fill");
            cur_w = vs[i].width;
        }
        p2r::FitLaunch a{n_tracks, n_layers, surf, trk, hits, out, chi2, st, nullptr};
        for (int w = 0; w < 2; ++w) TRY(p2r::launch_fit(vs[i], a, P, s), "kernel launch");
        TRY(hipEventRecord(e0, s), "hipEventRecord");
        const int reps = 5;
        for (int r = 0; r < reps; ++r) TRY(p2r::launch_fit(vs[i], a, P, s), "kernel launch");
        TRY(hipEventRecord(e1, s), "hipEventRecord");
        TRY(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (ms < best) { best = ms; best_i = (int)i; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
#undef TRY
    if (best_i < 0) return fail(P2R_ENOTUNED, "no variant for which=%d", which);
    ctx->chosen[which] = best_i;
    ctx->cache[key] = vs[best_i].name;
    save_cache(ctx);
    return P2R_OK;
}

}  // extern "C"
