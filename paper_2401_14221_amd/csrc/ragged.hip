// Ragged batched fit: every track has its own ordered list of surfaces
// (CSR), each a cylinder or a plane, with one 3D hit per surface.
//
// Schedule (all on the caller's stream, captured once into a HIP graph):
//   1. rag_reset   zero the key histogram and the work-queue counter
//   2. rag_hist    sort key of every track; per-workgroup histogram in LDS,
//                  then one global atomic per (workgroup, key)
//   3. rag_scan    (one workgroup) bucket starts, and for every block of
//                  RAG_W sorted tracks its first packed layer row
//   4. rag_scatter counting-sort scatter -> perm[sorted position] = track and
//                  run[sorted position] = its CSR run, ranks from LDS
//                  atomics, one cursor atomic per (workgroup, key)
//   5. rag_pack    one workgroup per block: copies its tracks' hits from the
//                  CSR arrays (coalesced reads of each track's run) through
//                  an LDS tile into [layer][RAG_FIELDS][RAG_W] rows
//   6. rag_fit_grid one wave per block, in block order: streams the block's
//                  packed rows (next layer prefetched) and fits its 64
//                  tracks (rag_fit: the same with a persistent grid whose
//                  waves take blocks from an atomic counter)
// The key orders tracks by surface count (longest first, so the longest
// blocks start first and the tail of the work is short blocks) and then by a
// |eta| bin, so the 64 lanes of a wave see similar surface sequences and
// branch the same way between cylinders and planes.  Gathering the hits
// lane by lane (each lane walking its own track's run) evicts each lane's
// cache lines before their next use, at 10-20x the algorithmic traffic; the
// pack pass reads every run with consecutive lanes instead.
#include "launch.h"
#include "track_math.h"

namespace p2r {

int ragged_nkeys(int lmax) { return (lmax + 1) * RAG_ETA_BINS + 1; }

int64_t ragged_packed_rows(int64_t n_hits, int lmax) {
    // sum over blocks of the block's (largest) surface count: a block inside
    // one key bucket holds RAG_W tracks of equal count; the last block and
    // each block that straddles a bucket boundary add at most lmax
    return (n_hits + RAG_W - 1) / RAG_W + (int64_t)lmax * ragged_nkeys(lmax) + 1;
}

__device__ __forceinline__ int track_key(const RaggedLaunch& a, int64_t t) {
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

// surface count of the tracks of sort key k (0 for the invalid bucket)
__device__ __forceinline__ int key_layers(const RaggedLaunch& a, int k) {
    return k >= a.nkeys - 1 ? 0 : a.lmax - k / RAG_ETA_BINS;
}

__global__ void rag_reset(RaggedLaunch a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nkeys) a.hist[i] = 0;
    if (i == 0) a.work[0] = 0;
}

// dynamic LDS: nkeys counters
__global__ void __launch_bounds__(256) rag_hist(RaggedLaunch a) {
    extern __shared__ int32_t lh[];
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x) lh[k] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * RAG_TPB;
    for (int i = threadIdx.x; i < RAG_TPB; i += blockDim.x) {
        const int64_t t = t0 + i;
        if (t < a.n) {
            const int key = track_key(a, t);
            a.keys[t] = key;
            atomicAdd(&lh[key], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x)
        if (lh[k]) atomicAdd(&a.hist[k], lh[k]);
}

// One workgroup of 1024 threads.  dynamic LDS: nkeys bucket starts.
//   base[k]    = sum of hist[k'] for k' < k
//   blk_off[b] = sum of Lb' for b' < b, Lb = surface count of the key bucket
//                holding the block's first sorted position (its largest,
//                since counts decrease along the sorted order); a block whose
//                rows would pass packed_cap gets none (its tracks are then
//                reported BAD_INPUT by the fit).
__global__ void __launch_bounds__(1024) rag_scan(RaggedLaunch a) {
    __shared__ int32_t part[1024];
    extern __shared__ int32_t sbase[];
    const int tid = threadIdx.x;
    {
        const int per = (a.nkeys + 1023) / 1024;
        const int lo = min(tid * per, a.nkeys), hi = min(lo + per, a.nkeys);
        int32_t s = 0;
        for (int i = lo; i < hi; ++i) s += a.hist[i];
        part[tid] = s;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t v = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        int32_t run = tid > 0 ? part[tid - 1] : 0;
        for (int i = lo; i < hi; ++i) {
            const int32_t c = a.hist[i];
            a.base[i] = run;
            sbase[i] = run;
            run += c;
        }
    }
    __syncthreads();
    // rows of block b: the bucket of position 64 b is the largest k with
    // sbase[k] <= 64 b (an empty bucket shares its start with the next one)
    auto rows_of = [&](int b) -> int {
        const int32_t pos = b * RAG_W;
        int lo = 0, hi = a.nkeys - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sbase[mid] <= pos) lo = mid; else hi = mid - 1;
        }
        return key_layers(a, lo);
    };
    const int per = (a.nb + 1023) / 1024;
    const int lo = min(tid * per, a.nb), hi = min(lo + per, a.nb);
    int64_t s = 0;
    for (int b = lo; b < hi; ++b) s += rows_of(b);
    __syncthreads();
    __shared__ int64_t part64[1024];
    part64[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? part64[tid - off] : 0;
        __syncthreads();
        part64[tid] += v;
        __syncthreads();
    }
    int64_t run = tid > 0 ? part64[tid - 1] : 0;
    const int64_t cap = a.packed_cap;
    for (int b = lo; b < hi; ++b) {
        const int r = rows_of(b);
        const int64_t start = run < cap ? run : cap;
        a.blk_off[b] = (int32_t)start;
        run += r;
    }
    if (tid == 1023) a.blk_off[a.nb] = (int32_t)(run < cap ? run : cap);
}

// dynamic LDS: 2 nkeys ints (ranks, workgroup bases)
__global__ void __launch_bounds__(256) rag_scatter(RaggedLaunch a) {
    extern __shared__ int32_t sh[];
    int32_t* lh = sh;
    int32_t* off = sh + a.nkeys;
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x) lh[k] = 0;
    __syncthreads();
    constexpr int PER = RAG_TPB / 256;
    int key[PER], rank[PER];
    const int64_t t0 = (int64_t)blockIdx.x * RAG_TPB;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + threadIdx.x + j * 256;
        key[j] = -1;
        if (t < a.n) {
            key[j] = a.keys[t];
            rank[j] = atomicAdd(&lh[key[j]], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x)
        if (lh[k]) off[k] = atomicAdd(&a.base[k], lh[k]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + threadIdx.x + j * 256;
        if (key[j] >= 0) {
            const int32_t pos = off[key[j]] + rank[j];
            a.perm[pos] = (int32_t)t;
            // the track's CSR run in sorted order, so that the pack and the
            // fit read it sequentially instead of gathering offsets[t]
            const int L = key_layers(a, key[j]);
            a.run[pos] = key[j] < a.nkeys - 1 ? (a.offsets[t] | ((int64_t)L << RAG_RUN_SHIFT)) : (int64_t)-1;
        }
    }
}

// One workgroup of 256 threads per block of RAG_W sorted tracks.  Row j of
// the block holds, for field f and the track at sorted position 64 b + l,
// packed[((blk_off[b] + j) RAG_FIELDS + f) RAG_W + l].  The rows are built in
// LDS tiles of up to PACK_ROWS rows for PACK_TRACKS tracks.  Filling a tile,
// the workgroup's threads cover each CSR array's runs of the tile's tracks
// with consecutive threads on consecutive elements (whole runs, so every
// fetched cache line is used), and each thread issues all of its loads
// (about 17) before it stores any of them, so that enough reads are in
// flight to cover the memory latency.  The tile is track-major with an odd
// track stride: the fill's stores and the drain's loads are free of bank
// conflicts.  It then goes out as 64-byte pieces of the block's rows, which
// the L2 merges into whole lines.  Tile entries of a track with fewer rows
// keep stale values, which the fit never reads (it stops at the track's
// count).
constexpr int PACK_ROWS = 24;
constexpr int PACK_TRACKS = 16;
constexpr int PACK_TSTRIDE = PACK_ROWS * RAG_FIELDS + 1;
constexpr int PACK_THREADS = 256;

__global__ void __launch_bounds__(PACK_THREADS) rag_pack(RaggedLaunch a) {
    __shared__ float tile[PACK_TRACKS * PACK_TSTRIDE];
    __shared__ int32_t s_rows[RAG_W];
    __shared__ int64_t s_h0[RAG_W];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t o = a.blk_off[b];
    const int rows = a.blk_off[b + 1] - (int32_t)o;
    if (tid < RAG_W) {
        const int64_t p = (int64_t)b * RAG_W + tid;
        int L = 0;
        int64_t h0 = 0;
        if (p < a.n) {
            const int64_t r = a.run[p];
            if (r >= 0) {                                // -1: invalid CSR range, no rows
                L = min((int)(r >> RAG_RUN_SHIFT), rows);
                h0 = r & (((int64_t)1 << RAG_RUN_SHIFT) - 1);
            }
        }
        s_rows[tid] = L;
        s_h0[tid] = h0;
    }
    __syncthreads();
    // per-track element counts of a full tile, and each thread's slots
    constexpr int NCOV = 6 * PACK_ROWS, NPOS = 3 * PACK_ROWS, NSUR = PACK_ROWS;
    constexpr int SC = (PACK_TRACKS * NCOV + PACK_THREADS - 1) / PACK_THREADS;
    constexpr int SP = (PACK_TRACKS * NPOS + PACK_THREADS - 1) / PACK_THREADS;
    constexpr int SS = (PACK_TRACKS * NSUR + PACK_THREADS - 1) / PACK_THREADS;
    float* dst = a.packed + (size_t)o * (RAG_FIELDS * RAG_W);
    __shared__ int32_t t_rows[PACK_TRACKS];              // rows of each tile track (<= 0: none)
    __shared__ int64_t t_h[PACK_TRACKS];                 // and its first hit in the tile
    for (int c0 = 0; c0 < rows; c0 += PACK_ROWS) {
        const int nr = min(PACK_ROWS, rows - c0);
        // The block's first track has the most rows (counts fall along the
        // sorted order), rows of them, so its hit c0 exists: slots that have
        // no element of their own load that one, which keeps every load
        // unconditional, and do not store it.
        const int64_t hsafe = s_h0[0] + c0;
        for (int k0 = 0; k0 < RAG_W; k0 += PACK_TRACKS) {
            if (tid < PACK_TRACKS) {
                t_rows[tid] = min(nr, s_rows[k0 + tid] - c0);
                t_h[tid] = s_h0[k0 + tid] + c0;
            }
            __syncthreads();
            // element index of every slot in its array (the safe one when idle)
            int64_t ic[SC], ip[SP], is[SS];
            bool okc[SC], okp[SP], oks[SS];
#pragma unroll
            for (int i = 0; i < SC; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = min(slot / NCOV, PACK_TRACKS - 1), e = slot - kt * NCOV;
                okc[i] = slot < PACK_TRACKS * NCOV && e < 6 * t_rows[kt];
                ic[i] = okc[i] ? t_h[kt] * 6 + e : hsafe * 6;
            }
#pragma unroll
            for (int i = 0; i < SP; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = min(slot / NPOS, PACK_TRACKS - 1), e = slot - kt * NPOS;
                okp[i] = slot < PACK_TRACKS * NPOS && e < 3 * t_rows[kt];
                ip[i] = okp[i] ? t_h[kt] * 3 + e : hsafe * 3;
            }
#pragma unroll
            for (int i = 0; i < SS; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = min(slot / NSUR, PACK_TRACKS - 1), e = slot - kt * NSUR;
                oks[i] = slot < PACK_TRACKS * NSUR && e < t_rows[kt];
                is[i] = oks[i] ? t_h[kt] + e : hsafe;
            }
            float vc[SC], vp[SP], vs[SS], vt[SS];
#pragma unroll
            for (int i = 0; i < SC; ++i) vc[i] = a.hcov[ic[i]];
#pragma unroll
            for (int i = 0; i < SP; ++i) vp[i] = a.hpos[ip[i]];
#pragma unroll
            for (int i = 0; i < SS; ++i) {
                vs[i] = a.sval[is[i]];
                vt[i] = (float)a.stype[is[i]];
            }
#pragma unroll
            for (int i = 0; i < SC; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = slot / NCOV, e = slot - kt * NCOV;
                if (okc[i]) tile[kt * PACK_TSTRIDE + (e / 6) * RAG_FIELDS + 5 + e % 6] = vc[i];
            }
#pragma unroll
            for (int i = 0; i < SP; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = slot / NPOS, e = slot - kt * NPOS;
                if (okp[i]) tile[kt * PACK_TSTRIDE + (e / 3) * RAG_FIELDS + 2 + e % 3] = vp[i];
            }
#pragma unroll
            for (int i = 0; i < SS; ++i) {
                const int slot = tid + PACK_THREADS * i, kt = slot / NSUR, e = slot - kt * NSUR;
                if (oks[i]) {
                    tile[kt * PACK_TSTRIDE + e * RAG_FIELDS + 1] = vs[i];
                    tile[kt * PACK_TSTRIDE + e * RAG_FIELDS] = vt[i];
                }
            }
            __syncthreads();
            float* d = dst + (size_t)c0 * (RAG_FIELDS * RAG_W) + k0;
            for (int e = tid; e < nr * RAG_FIELDS * PACK_TRACKS; e += PACK_THREADS) {
                const int rf = e / PACK_TRACKS, kt = e % PACK_TRACKS;   // rf = row * RAG_FIELDS + field
                d[(size_t)rf * RAG_W + kt] = tile[kt * PACK_TSTRIDE + rf];
            }
            __syncthreads();
        }
    }
}

// Fits the track at sorted position RAG_W b + lane (b uniform over the
// wave).  Every load the block needs first (its rows, the track record, the
// first packed row) is issued before any is used, so the block start costs
// one memory round trip after the perm/run reads.
template <typename T, bool U2D>
__device__ __forceinline__ void fit_sorted_track(const RaggedLaunch& a, const Params& P, int b, int lane) {
    const int64_t p = (int64_t)b * RAG_W + lane;
    const bool live = p < a.n;                    // lane 0 always is
    const int64_t o = a.blk_off[b];
    const int rows = a.blk_off[b + 1] - (int32_t)o;
    // run[p]: the surface count of a track whose CSR range the sort found
    // valid (0 <= L <= lmax, inside [0, n_hits)); -1 for every other track.
    // A lane past the last track reads the last track's entries, which it
    // never uses (no branch around the loads).
    const int64_t pc = live ? p : (int64_t)a.n - 1;
    const int t = a.perm[pc];
    const int64_t r = live ? a.run[pc] : (int64_t)-1;
    StateT<T> st;
#pragma unroll
    for (int f = 0; f < 6; ++f) st.p[f] = a.par_in[(size_t)t * 6 + f];
#pragma unroll
    for (int f = 0; f < 21; ++f) st.c[f] = a.cov_in[(size_t)t * 21 + f];
    const int qi = a.q[t];
    st.q = (T)qi;
    const float* src = a.packed + (size_t)o * (RAG_FIELDS * RAG_W) + lane;
    float hb[RAG_FIELDS];
    if (rows > 0) {
#pragma unroll
        for (int f = 0; f < RAG_FIELDS; ++f) hb[f] = src[f * RAG_W];
    }
    if (!live) return;
    const int L = r < 0 ? 0 : (int)(r >> RAG_RUN_SHIFT);
    uint32_t flags = 0;
    int nused = 0;
    T chi2 = 0;
    const bool bad = (r < 0) | (L > rows) | ((qi != 1) & (qi != -1)) | bad_input(st);
    if (bad) {
        flags = ST_BAD_INPUT;
    } else {
        for (int j = 0; j < (int)L; ++j) {
            const float type = hb[0];
            const T v = hb[1];
            const T m[3] = {hb[2], hb[3], hb[4]};
            const T V[6] = {hb[5], hb[6], hb[7], hb[8], hb[9], hb[10]};
            if (j + 1 < (int)L) {
                const float* nx = src + (size_t)(j + 1) * (RAG_FIELDS * RAG_W);
#pragma unroll
                for (int f = 0; f < RAG_FIELDS; ++f) hb[f] = nx[f * RAG_W];
            }
            T c2 = 0;
            StepOut out{0u, false, 0};
            if constexpr (U2D) {
                // cylinders and planes take different updates
                if (type == 0.0f) out = step_cylinder<T, true>(st, v, m, V, P, c2, newton_tol(P.tol, v), T(NAN));
                else if (type == 1.0f) out = step_plane<T>(st, v, m, V, P, c2);
                else out.flags = ST_BAD_INPUT;
            } else {
                // Lanes of one wave may meet cylinders and planes in the same
                // row: the two propagations diverge, and the update after them
                // is shared, so such a row costs one update, not two.
                if (type == 0.0f) out = step_cylinder<T, false, false>(st, v, m, V, P, c2, newton_tol(P.tol, v), T(NAN));
                else if (type == 1.0f) out = step_plane<T, false>(st, v, m, V, P, c2);
                else out.flags = ST_BAD_INPUT;
                if (out.updated) update_step<T>(st, m, V, P, c2, out);
            }
            flags |= out.flags;
            if (out.updated) { ++nused; chi2 += c2; }
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) a.par_out[(size_t)t * 6 + f] = (float)st.p[f];
#pragma unroll
    for (int f = 0; f < 21; ++f) a.cov_out[(size_t)t * 21 + f] = (float)st.c[f];
    a.chi2[t] = (float)chi2;
    a.status[t] = flags | ST_DONE | ((uint32_t)(nused > 255 ? 255 : nused) << NUSED_SHIFT);
}

// The fit, one workgroup (one wave) per block of RAG_W sorted tracks: the
// dispatcher hands the blocks out in order, longest first, and refills each
// slot as its wave ends.  (Faster here than the persistent work queue below:
// 0.96 against 1.07 ms for the 10^6-track ragged workload.)
template <int WPE, typename T, bool U2D>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
rag_fit_grid(RaggedLaunch a, Params P) {
    fit_sorted_track<T, U2D>(a, P, blockIdx.x, threadIdx.x);
}

// The persistent variant: a grid of resident waves takes blocks from an
// atomic counter.  Every wave leaves the loop once the counter passes the
// last block, so the grid drains whatever its size.
template <int WPE, typename T, bool U2D>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
rag_fit(RaggedLaunch a, Params P) {
    const int lane = threadIdx.x;
    while (true) {
        int b = 0;
        if (lane == 0) b = atomicAdd(a.work, 1);
        b = __builtin_amdgcn_readfirstlane(b);
        if (b >= a.nb) break;
        fit_sorted_track<T, U2D>(a, P, b, lane);
    }
}

template __global__ void rag_fit_grid<0, float, false>(RaggedLaunch, Params);
template __global__ void rag_fit_grid<2, double, false>(RaggedLaunch, Params);
template __global__ void rag_fit_grid<4, float, true>(RaggedLaunch, Params);
template __global__ void rag_fit_grid<2, double, true>(RaggedLaunch, Params);
template __global__ void rag_fit<0, float, false>(RaggedLaunch, Params);
template __global__ void rag_fit<4, float, false>(RaggedLaunch, Params);

// FP32 at occupancy target wpe (0 or 4), or FP64; the 3D update or the one
// in the hit frame on cylinders (128 VGPRs, spilling only at the FP64 calls)
const void* ragged_grid_symbol(bool fp64, bool u2d) {
    if (fp64) return u2d ? (const void*)&rag_fit_grid<2, double, true> : (const void*)&rag_fit_grid<2, double, false>;
    return u2d ? (const void*)&rag_fit_grid<4, float, true> : (const void*)&rag_fit_grid<0, float, false>;
}

const void* ragged_fit_symbol(int wpe) {
    return wpe == 4 ? (const void*)&rag_fit<4, float, false> : (const void*)&rag_fit<0, float, false>;
}

hipError_t launch_ragged(const Variant& v, const RaggedLaunch& a, const Params& P, hipStream_t s) {
    RaggedLaunch aa = a;
    Params pp = P;
    const int tb = 256;
    const size_t lds_keys = sizeof(int32_t) * (size_t)a.nkeys;
    hipLaunchKernelGGL(rag_reset, dim3((a.nkeys + tb - 1) / tb), dim3(tb), 0, s, aa);
    const int64_t nwg = ((int64_t)a.n + RAG_TPB - 1) / RAG_TPB;
    if (nwg > 0) {
        hipLaunchKernelGGL(rag_hist, dim3((unsigned)nwg), dim3(tb), lds_keys, s, aa);
        hipLaunchKernelGGL(rag_scan, dim3(1), dim3(1024), lds_keys, s, aa);
        hipLaunchKernelGGL(rag_scatter, dim3((unsigned)nwg), dim3(tb), 2 * lds_keys, s, aa);
        hipLaunchKernelGGL(rag_pack, dim3(a.nb), dim3(PACK_THREADS), 0, s, aa);
        void* args[] = {&aa, &pp};
        hipError_t e = hipLaunchKernel(v.fn, dim3(v.per_block ? a.nb : a.grid), dim3(RAG_W), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace p2r
