// Ragged batched fit: every track has its own ordered list of surfaces
// (CSR), each a cylinder or a plane, with one 3D hit per surface.
//
// Schedule (all on the caller's stream, captured once into a HIP graph):
//   1. rag_reset   zero the key histogram and the work-queue counter
//   2. rag_hist    sort key of every track -> histogram (wave-aggregated atomics)
//   3. rag_scan    exclusive scan of the histogram (one workgroup)
//   4. rag_scatter counting-sort scatter -> perm[sorted position] = track
//   5. rag_fit     persistent kernel: each wave takes the next block of 64
//                  sorted tracks from an atomic counter until none is left
// The key orders tracks by surface count (longest first, so the longest
// blocks start first and the tail of the queue is short work) and then by a
// |eta| bin, so the 64 lanes of a wave see similar surface sequences and
// branch the same way between cylinders and planes.
#include "launch.h"
#include "track_math.h"

namespace p2r {

int ragged_nkeys(int lmax) { return (lmax + 1) * RAG_ETA_BINS + 1; }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// atomicAdd(&ctr[key], 1) for every lane with pred, aggregated per distinct
// key within the wave; returns the lane's slot (old value + rank).
__device__ __forceinline__ int aggregated_inc(int32_t* ctr, int key, bool pred) {
    uint64_t todo = __ballot(pred);
    const int lane = lane_id();
    int ret = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int lkey = __shfl(key, leader);
        const uint64_t grp = __ballot(pred && key == lkey) & todo;
        int old = 0;
        if (lane == leader) old = atomicAdd(&ctr[lkey], __popcll(grp));
        old = __shfl(old, leader);
        if ((grp >> lane) & 1ull) ret = old + __popcll(grp & ((1ull << lane) - 1ull));
        todo &= ~grp;
    }
    return ret;
}

__device__ __forceinline__ int track_key(const RaggedLaunch& a, int t) {
    const int64_t h0 = a.offsets[t];
    const int64_t L = a.offsets[t + 1] - h0;
    const int invalid = a.nkeys - 1;
    if (L < 0 || L > a.lmax || h0 < 0 || h0 + L > a.n_hits) return invalid;
    const float th = a.par_in[(size_t)t * 6 + 5];
    if (!(th > 0.0f && th < PI_F)) return invalid;
    const float aeta = asinhf(fabsf(cosf(th) / sinf(th)));
    int bin = (int)(aeta * (RAG_ETA_BINS / 2.5f));
    bin = bin < 0 ? 0 : (bin >= RAG_ETA_BINS ? RAG_ETA_BINS - 1 : bin);
    return (a.lmax - (int)L) * RAG_ETA_BINS + bin;
}

__global__ void rag_reset(RaggedLaunch a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nkeys) a.hist[i] = 0;
    if (i == 0) a.work[0] = 0;
}

__global__ void rag_hist(RaggedLaunch a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = t < a.n;
    const int key = ok ? track_key(a, t) : 0;
    if (ok) a.keys[t] = key;
    (void)aggregated_inc(a.hist, key, ok);
}

// exclusive scan of hist[0..nkeys) in place, one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) rag_scan(RaggedLaunch a) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (a.nkeys + 1023) / 1024;
    const int lo = tid * per;
    const int hi = min(lo + per, a.nkeys);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a.hist[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = tid > 0 ? part[tid - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        int32_t c = a.hist[i];
        a.hist[i] = run;
        run += c;
    }
}

__global__ void rag_scatter(RaggedLaunch a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = t < a.n;
    const int key = ok ? a.keys[t] : 0;
    const int pos = aggregated_inc(a.hist, key, ok);
    if (ok) a.perm[pos] = t;
}

__device__ __forceinline__ void fit_ragged_track(const RaggedLaunch& a, const Params& P, int t) {
    State st;
#pragma unroll
    for (int f = 0; f < 6; ++f) st.p[f] = a.par_in[(size_t)t * 6 + f];
#pragma unroll
    for (int f = 0; f < 21; ++f) st.c[f] = a.cov_in[(size_t)t * 21 + f];
    const int qi = a.q[t];
    st.q = (float)qi;
    const int64_t h0 = a.offsets[t];
    const int64_t L = a.offsets[t + 1] - h0;
    uint32_t flags = 0;
    int nused = 0;
    float chi2 = 0.0f;
    if (L < 0 || L > a.lmax || h0 < 0 || h0 + L > a.n_hits || (qi != 1 && qi != -1) || bad_input(st)) {
        flags = ST_BAD_INPUT;
    } else {
        for (int j = 0; j < (int)L; ++j) {
            const int64_t h = h0 + j;
            const int type = a.stype[h];
            const float v = a.sval[h];
            const float m[3] = {a.hpos[h * 3], a.hpos[h * 3 + 1], a.hpos[h * 3 + 2]};
            float V[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) V[k] = a.hcov[h * 6 + k];
            float c2 = 0.0f;
            StepOut o;
            if (type == 0) {
                o = step_cylinder(st, v, m, V, P, c2, newton_tol(P.tol, v), NAN);
            } else if (type == 1) {
                o = step_plane(st, v, m, V, P, c2);
            } else {
                o = StepOut{ST_BAD_INPUT, false, 0};
            }
            flags |= o.flags;
            if (o.updated) { ++nused; chi2 += c2; }
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) a.par_out[(size_t)t * 6 + f] = st.p[f];
#pragma unroll
    for (int f = 0; f < 21; ++f) a.cov_out[(size_t)t * 21 + f] = st.c[f];
    a.chi2[t] = chi2;
    a.status[t] = flags | ST_DONE | ((uint32_t)(nused > 255 ? 255 : nused) << NUSED_SHIFT);
}

// Every wave leaves the loop once the counter passes the last block, so the
// grid drains whatever its size.
template <int WPE>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
rag_fit(RaggedLaunch a, Params P) {
    const int lane = threadIdx.x;
    while (true) {
        int b = 0;
        if (lane == 0) b = atomicAdd(a.work, 1);
        b = __shfl(b, 0);
        if (b >= a.nb) break;
        const int k = b * RAG_W + lane;
        if (k < a.n) fit_ragged_track(a, P, a.perm[k]);
    }
}

template __global__ void rag_fit<0>(RaggedLaunch, Params);
template __global__ void rag_fit<4>(RaggedLaunch, Params);

const void* ragged_fit_symbol(int wpe) {
    return wpe == 4 ? (const void*)&rag_fit<4> : (const void*)&rag_fit<0>;
}

hipError_t launch_ragged(const Variant& v, const RaggedLaunch& a, const Params& P, hipStream_t s) {
    RaggedLaunch aa = a;
    Params pp = P;
    const int tb = 256;
    hipLaunchKernelGGL(rag_reset, dim3((a.nkeys + tb - 1) / tb), dim3(tb), 0, s, aa);
    const int nbt = (a.n + tb - 1) / tb;
    if (nbt > 0) {
        hipLaunchKernelGGL(rag_hist, dim3(nbt), dim3(tb), 0, s, aa);
        hipLaunchKernelGGL(rag_scan, dim3(1), dim3(1024), 0, s, aa);
        hipLaunchKernelGGL(rag_scatter, dim3(nbt), dim3(tb), 0, s, aa);
        void* args[] = {&aa, &pp};
        hipError_t e = hipLaunchKernel(v.fn, dim3(a.grid), dim3(RAG_W), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace p2r
