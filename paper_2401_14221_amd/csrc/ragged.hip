// Ragged batched fit: every track has its own ordered list of surfaces
// (CSR), each a cylinder or a plane, with one 3D hit per surface.
//
// Schedule (all on the caller's stream, captured once into a HIP graph):
//   1. rag_reset   zero the key histogram, the key cursors and the
//                  work-queue counter
//   2. rag_hist    sort key of every track; per-workgroup histogram in LDS,
//                  then one global atomic per (workgroup, key)
//   3. rag_scatter counting-sort scatter -> perm[sorted position] = track and
//                  run[sorted position] = its CSR run: every workgroup takes
//                  the first sorted position of each key from a prefix sum
//                  of the (small) histogram in LDS, its tracks' ranks from
//                  LDS atomics, and one cursor atomic per (workgroup, key)
//   4. rag_fit_*   one wave per block of RAG_W sorted tracks: streams the
//                  block's hits from the CSR arrays through LDS, a chunk of
//                  surfaces at a time, and fits its 64 tracks (the queue
//                  variant: a persistent grid whose waves take blocks from an
//                  atomic counter)
// The key orders tracks by surface count (longest first, so the longest
// blocks start first and the tail of the work is short blocks) and then by a
// |eta| bin, so the 64 lanes of a wave see similar surface sequences and
// branch the same way between cylinders and planes.  Gathering the hits
// lane by lane (each lane walking its own track's run) would evict each
// lane's cache lines before their next use; the staged copy reads the runs
// with consecutive lanes instead.
#include "launch.h"
#include "track_math.h"

namespace p2r {

int ragged_nkeys(int lmax) { return (lmax + 1) * RAG_ETA_BINS + 1; }

// The sort key of a track from its CSR offsets h0 = offsets[t],
// h1 = offsets[t + 1] and its theta.
__device__ __forceinline__ int track_key(const RaggedLaunch& a, int64_t h0, int64_t h1, float th) {
    const int64_t L = h1 - h0;
    const int invalid = a.nkeys - 1;
    if (L < 0 || L > a.lmax || h0 < 0 || h0 + L > a.n_hits) return invalid;
    if (!(th > 0.0f && th < PI_F)) return invalid;
    // |eta| bin of width 2.5 / RAG_ETA_BINS, from |cos theta| = tanh|eta|
    // against the bin edges tanh(k 2.5 / 8) (the bin only groups tracks, so
    // the fast cosine's error at an edge does not matter)
    static_assert(RAG_ETA_BINS == 8, "bin edges below are for 8 bins of 0.3125");
    const float c = fabsf(__cosf(th));
    const int bin = (c >= 0.302709729f) + (c >= 0.554599722f) + (c >= 0.73407152f) + (c >= 0.84828364f) +
                    (c >= 0.915824544f) + (c >= 0.95404526f) + (c >= 0.975136698f);
    return (a.lmax - (int)L) * RAG_ETA_BINS + bin;
}

// surface count of the tracks of sort key k (0 for the invalid bucket)
__device__ __forceinline__ int key_layers(const RaggedLaunch& a, int k) {
    return k >= a.nkeys - 1 ? 0 : a.lmax - k / RAG_ETA_BINS;
}

__global__ void rag_reset(RaggedLaunch a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nkeys) {
        a.hist[i] = 0;
        a.base[i] = 0;
    }
    if (i == 0) a.work[0] = 0;
}

// dynamic LDS: nkeys counters
__global__ void __launch_bounds__(256) rag_hist(RaggedLaunch a) {
    extern __shared__ int32_t lh[];
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x) lh[k] = 0;
    __syncthreads();
    // every load first: a load placed after a key store (which might alias
    // it, for all the compiler knows) would wait for that store
    constexpr int PER = RAG_TPB / 256;
    const int64_t t0 = (int64_t)blockIdx.x * RAG_TPB;
    int64_t h0[PER], h1[PER];
    float th[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + threadIdx.x + j * 256;
        if (t < a.n) {
            h0[j] = a.offsets[t];
            h1[j] = a.offsets[t + 1];
            th[j] = a.par_in[(size_t)t * 6 + 5];
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + threadIdx.x + j * 256;
        if (t < a.n) {
            const int key = track_key(a, h0[j], h1[j], th[j]);
            a.keys[t] = key;
            atomicAdd(&lh[key], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < a.nkeys; k += blockDim.x)
        if (lh[k]) atomicAdd(&a.hist[k], lh[k]);
}

// dynamic LDS: 3 nkeys ints (ranks, first sorted positions, workgroup bases)
// plus 256 partial sums.  base[] holds the keys' cursors (zeroed by
// rag_reset): a workgroup's tracks of key k go to first[k] + the cursor's
// value before its atomic add.
__global__ void __launch_bounds__(256) rag_scatter(RaggedLaunch a) {
    extern __shared__ int32_t sh[];
    int32_t* lh = sh;
    int32_t* off = sh + a.nkeys;
    int32_t* first = sh + 2 * a.nkeys;
    int32_t* part = sh + 3 * a.nkeys;
    const int tid = threadIdx.x;
    // exclusive prefix sum of the finished histogram: thread tid sums a
    // contiguous range of keys, the 256 range sums are scanned in LDS, then
    // each thread writes its range's first positions
    const int per = (a.nkeys + 255) / 256;
    const int lo = min(tid * per, a.nkeys), hi = min(lo + per, a.nkeys);
    int32_t sum = 0;
    for (int k = lo; k < hi; ++k) {
        const int32_t c = a.hist[k];
        first[k] = sum;
        sum += c;
        lh[k] = 0;
    }
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const int32_t before = tid > 0 ? part[tid - 1] : 0;
    for (int k = lo; k < hi; ++k) first[k] += before;
    __syncthreads();
    constexpr int PER = RAG_TPB / 256;
    int key[PER], rank[PER];
    int64_t h0[PER];
    const int64_t t0 = (int64_t)blockIdx.x * RAG_TPB;
    // the keys and CSR offsets are loaded before any store (see rag_hist)
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + tid + j * 256;
        key[j] = -1;
        if (t < a.n) {
            key[j] = a.keys[t];
            h0[j] = a.offsets[t];
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if (key[j] >= 0) rank[j] = atomicAdd(&lh[key[j]], 1);
    __syncthreads();
    for (int k = tid; k < a.nkeys; k += blockDim.x)
        if (lh[k]) off[k] = first[k] + atomicAdd(&a.base[k], lh[k]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t t = t0 + tid + j * 256;
        if (key[j] >= 0) {
            const int32_t pos = off[key[j]] + rank[j];
            a.perm[pos] = (int32_t)t;
            // the track's CSR run in sorted order, so that the fit reads it
            // sequentially instead of gathering offsets[t]
            const int L = key_layers(a, key[j]);
            a.run[pos] = key[j] < a.nkeys - 1 ? (h0[j] | ((int64_t)L << RAG_RUN_SHIFT)) : (int64_t)-1;
        }
    }
}

// ------------------------------------------------------------ the fit
// One wave fits the RAG_W tracks at sorted positions RAG_W b .. RAG_W b + 63,
// lane l the track at RAG_W b + l.  The wave streams the tracks' hits through
// LDS: it copies a chunk of surfaces of its 64 tracks from the CSR arrays
// into rows [surface][field][lane], then each lane reads its own hits from
// there.  The copy is coalesced: for each CSR array the 64 tracks' runs of
// the chunk's surfaces are read by consecutive lanes on consecutive
// elements, so a load instruction touches a few cache lines instead of 64.
// A cache line that holds the end of one chunk of a track and the start of
// its next is evicted from L2 before the next chunk is read (the wave's next
// chunk comes tens of microseconds later), so every chunk read costs about
// one extra line per array and track.  The small arrays (surface type and
// value, 5 B per surface) are therefore read in chunks of CB surfaces, the
// hit position and covariance (36 B per surface) in chunks of C, which is
// what bounds the LDS a wave needs.  Every load of a chunk is issued before
// any is stored (PREFETCH: the next chunk's loads are issued before the
// current chunk is fitted, and stored after it).  Tracks are sorted by
// surface count, longest first, so the block's first track has the most
// surfaces and a wave needs as many chunks as that track.

constexpr int RAG_HIT_FIELDS = 9;      // hit position (3) and covariance (6)

// Staging area of one wave: the rows of the current chunks, and each lane's
// CSR run (first hit, surface count; count 0 for a track that is not fitted).
template <int C, int CB>
struct RagStage {
    float hit[C * RAG_HIT_FIELDS * RAG_LSTRIDE];   // [j][field][lane], surfaces k0 .. k0 + C - 1
    float sval[CB * RAG_LSTRIDE];                  // [j][lane], surfaces kb .. kb + CB - 1
    uint8_t stype[CB * RAG_W];                     // [j][lane]
    uint2 run[RAG_W];
};

// Which element of a chunk of K surfaces each lane copies.  Lane l serves
// the tracks tt = g (64 / K) + l / K, g = 0 .. K - 1, as sub-lane u = l % K
// of each: of a track's K E units in an array with E units per surface (the
// run of its surfaces k0 .. k0 + K - 1), sub-lane u takes units u, u + K,
// ..., u + (E - 1) K, so the K sub-lanes of a track read consecutive units
// and a load instruction covers 64 / K tracks.  A unit past the track's last
// surface is not copied: its slot loads unit 0 of the array (which exists
// whenever any track has a surface) and stores nothing.
template <int K>
struct Lanes {
    uint32_t h0[K];    // CSR index of surface k0 of each served track
    int cnt[K];        // its surfaces left from k0 on
    int tt[K];         // its lane in the block
    int u;             // sub-lane
};

template <int K>
__device__ __forceinline__ Lanes<K> lanes_of(const uint2* run, int lane, int k0) {
    Lanes<K> q;
    q.u = lane % K;
#pragma unroll
    for (int g = 0; g < K; ++g) {
        q.tt[g] = g * (RAG_W / K) + lane / K;
        const uint2 r = run[q.tt[g]];
        q.h0[g] = r.x + (uint32_t)k0;
        q.cnt[g] = (int)r.y - k0;
    }
    return q;
}

// unit m (0 .. E - 1) of sub-lane u for served track g: surface j of the
// chunk, and the unit's index in its array (0 when it is past the run)
template <int K, int E>
__device__ __forceinline__ uint32_t unit_src(const Lanes<K>& q, int g, int m, int& j, bool& ok) {
    const int unit = q.u + K * m;
    j = unit / E;
    ok = j < q.cnt[g];
    return ok ? q.h0[g] * E + (uint32_t)unit : 0u;
}

// Loads of one chunk, held in registers between issue and store.
template <int C>
struct HitRegs {
    float p[3 * C];         // hit position, one float per slot
    float2 c[3 * C];        // hit covariance, two floats per slot
};
template <int CB>
struct SurfRegs {
    uint32_t t[CB];         // surface type byte
    float v[CB];            // surface value
};

// The slot arithmetic depends only on the lane and the chunk, so the
// compiler would hoist it out of the chunk loop and keep ~2 registers per
// slot alive through the whole fit; a lane index it cannot see through keeps
// it where it is used.
__device__ __forceinline__ int opaque_lane(int lane) {
    asm volatile("" : "+v"(lane));
    return lane;
}

// Wait until every vector memory load this wave issued has landed.  A slot
// past a track's run is loaded but never stored, and the compiler's wait
// tracking keeps such a load pending: a register it wrote and the fit later
// reuses would then need a wait inside the fit loop, which the in-order load
// counter turns into a wait for the whole prefetch issued after it.  Taken
// once per chunk, after the stores, where every load has landed anyway.
__device__ __forceinline__ void loads_landed() {
    // s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima (7, 15)
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Element i of an array at a 32-bit byte offset from its base (the call
// checks that every CSR array stays below 4 GiB), so that each load needs one
// offset register rather than a 64-bit address.
template <typename V>
__device__ __forceinline__ V load_at(const void* base, uint32_t i) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(V));
}

template <int C>
__device__ __forceinline__ void hit_load(const RaggedLaunch& a, const uint2* run, int lane, int k0, HitRegs<C>& R) {
    const Lanes<C> q = lanes_of<C>(run, opaque_lane(lane), k0);
    int j;
    bool ok;
#pragma unroll
    for (int g = 0; g < C; ++g)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            R.p[3 * g + m] = load_at<float>(a.hpos, unit_src<C, 3>(q, g, m, j, ok));
            R.c[3 * g + m] = load_at<float2>(a.hcov, unit_src<C, 3>(q, g, m, j, ok));
        }
}

template <int C, int CB>
__device__ __forceinline__ void hit_store(RagStage<C, CB>& S, int lane, int k0, const HitRegs<C>& R) {
    const Lanes<C> q = lanes_of<C>(S.run, opaque_lane(lane), k0);
    int j;
    bool ok;
#pragma unroll
    for (int g = 0; g < C; ++g)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            (void)unit_src<C, 3>(q, g, m, j, ok);
            const int e = q.u + C * m - 3 * j;          // position / covariance pair within the surface
            if (ok) {
                float* row = S.hit + j * (RAG_HIT_FIELDS * RAG_LSTRIDE) + q.tt[g];
                row[e * RAG_LSTRIDE] = R.p[3 * g + m];
                row[(3 + 2 * e) * RAG_LSTRIDE] = R.c[3 * g + m].x;
                row[(4 + 2 * e) * RAG_LSTRIDE] = R.c[3 * g + m].y;
            }
        }
}

template <int CB>
__device__ __forceinline__ void surf_load(const RaggedLaunch& a, const uint2* run, int lane, int k0, SurfRegs<CB>& R) {
    const Lanes<CB> q = lanes_of<CB>(run, opaque_lane(lane), k0);
    int j;
    bool ok;
#pragma unroll
    for (int g = 0; g < CB; ++g) {
        R.t[g] = load_at<uint8_t>(a.stype, unit_src<CB, 1>(q, g, 0, j, ok));
        R.v[g] = load_at<float>(a.sval, unit_src<CB, 1>(q, g, 0, j, ok));
    }
}

template <int C, int CB>
__device__ __forceinline__ void surf_store(RagStage<C, CB>& S, int lane, int k0, const SurfRegs<CB>& R) {
    const Lanes<CB> q = lanes_of<CB>(S.run, opaque_lane(lane), k0);
    int j;
    bool ok;
#pragma unroll
    for (int g = 0; g < CB; ++g) {
        (void)unit_src<CB, 1>(q, g, 0, j, ok);
        if (ok) {
            S.stype[j * RAG_W + q.tt[g]] = (uint8_t)R.t[g];
            S.sval[j * RAG_LSTRIDE + q.tt[g]] = R.v[g];
        }
    }
}

template <int C, int CB, bool PREFETCH, typename T, bool U2D>
__device__ __forceinline__ void fit_block(const RaggedLaunch& a, const Params& P, RagStage<C, CB>& S, int b, int lane) {
    static_assert(CB % C == 0 && RAG_W % CB == 0 && RAG_W % C == 0, "chunk sizes");
    const int64_t p = (int64_t)b * RAG_W + lane;
    const bool live = p < a.n;                    // lane 0 always is
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
    const int L = r < 0 ? 0 : (int)(r >> RAG_RUN_SHIFT);
    const bool bad = (r < 0) | ((qi != 1) & (qi != -1)) | bad_input(st);
    // the previous block's wave may still read the staging area
    __syncthreads();
    S.run[lane] = make_uint2((uint32_t)(r & (((int64_t)1 << RAG_RUN_SHIFT) - 1)), bad ? 0u : (uint32_t)L);
    // surfaces to stage: the block's first track has the most
    const int rows = __builtin_amdgcn_readfirstlane(L);
    uint32_t flags = bad ? ST_BAD_INPUT : 0u;
    int nused = 0;
    T chi2 = 0;
    HitRegs<C> RH;
    __syncthreads();
    if (rows > 0) hit_load<C>(a, S.run, lane, 0, RH);
    for (int k0 = 0; k0 < rows; k0 += C) {
        const int kb = k0 % CB;                 // this chunk's first row in the CB rows
        __syncthreads();                        // lanes are done reading the previous chunk
        hit_store<C, CB>(S, lane, k0, RH);
        if (kb == 0) {
            // the surface types and values of CB surfaces, loaded and stored
            // at once (after the hit registers are free) so that their
            // registers are free during the fit; the wait is taken once
            // every CB surfaces
            SurfRegs<CB> RS;
            surf_load<CB>(a, S.run, lane, k0, RS);
            surf_store<C, CB>(S, lane, k0, RS);
        }
        loads_landed();
        __syncthreads();
        const int k1 = k0 + C;
        if (PREFETCH && k1 < rows) hit_load<C>(a, S.run, lane, k1, RH);
        const int nj = bad ? 0 : min(C, L - k0);
#pragma unroll 1
        for (int j = 0; j < nj; ++j) {
            const float* row = S.hit + j * (RAG_HIT_FIELDS * RAG_LSTRIDE) + lane;
            float hb[RAG_HIT_FIELDS];
#pragma unroll
            for (int f = 0; f < RAG_HIT_FIELDS; ++f) hb[f] = row[f * RAG_LSTRIDE];
            const int type = S.stype[(kb + j) * RAG_W + lane];
            const T v = S.sval[(kb + j) * RAG_LSTRIDE + lane];
            const T m[3] = {hb[0], hb[1], hb[2]};
            const T V[6] = {hb[3], hb[4], hb[5], hb[6], hb[7], hb[8]};
            T c2 = 0;
            StepOut out{0u, false, 0};
            if constexpr (U2D) {
                // cylinders and planes take different updates
                if (type == 0) out = step_cylinder<T, true>(st, v, m, V, P, c2, newton_tol(P.tol, v), T(NAN));
                else if (type == 1) out = step_plane<T>(st, v, m, V, P, c2);
                else out.flags = ST_BAD_INPUT;
            } else {
                // Lanes of one wave may meet cylinders and planes in the same
                // row: the two propagations diverge, and the update after them
                // is shared, so such a row costs one update, not two.
                if (type == 0) out = step_cylinder<T, false, false>(st, v, m, V, P, c2, newton_tol(P.tol, v), T(NAN));
                else if (type == 1) out = step_plane<T, false>(st, v, m, V, P, c2);
                else out.flags = ST_BAD_INPUT;
                if (out.updated) update_step<T>(st, m, V, P, c2, out, type);
            }
            flags |= out.flags;
            if (out.updated) { ++nused; chi2 += c2; }
        }
        if (!PREFETCH && k1 < rows) hit_load<C>(a, S.run, lane, k1, RH);
    }
    if (!live) return;
    finalise(st);
#pragma unroll
    for (int f = 0; f < 6; ++f) a.par_out[(size_t)t * 6 + f] = (float)st.p[f];
#pragma unroll
    for (int f = 0; f < 21; ++f) a.cov_out[(size_t)t * 21 + f] = (float)st.c[f];
    a.chi2[t] = (float)chi2;
    a.status[t] = flags | ST_DONE | nused_field(nused);
}

// One workgroup (one wave) per block: the dispatcher hands the blocks out in
// order, longest first, and refills each slot as its wave ends.
template <int C, int CB, bool PREFETCH, int WPE, typename T, bool U2D>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
rag_fit_grid(RaggedLaunch a, Params P) {
    __shared__ RagStage<C, CB> S;
    fit_block<C, CB, PREFETCH, T, U2D>(a, P, S, blockIdx.x, threadIdx.x);
}

// The persistent variant: a grid of resident waves takes blocks from an
// atomic counter.  Every wave leaves the loop once the counter passes the
// last block, so the grid drains whatever its size.
template <int C, int CB, bool PREFETCH, int WPE, typename T, bool U2D>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
rag_fit_queue(RaggedLaunch a, Params P) {
    __shared__ RagStage<C, CB> S;
    const int lane = threadIdx.x;
    while (true) {
        int b = 0;
        if (lane == 0) b = atomicAdd(a.work, 1);
        b = __builtin_amdgcn_readfirstlane(b);
        if (b >= a.nb) break;
        fit_block<C, CB, PREFETCH, T, U2D>(a, P, S, b, lane);
    }
}

#define RAG_GRID(C, CB, PF, WPE, T, U2D) (const void*)&rag_fit_grid<C, CB, PF, WPE, T, U2D>
#define RAG_QUEUE(C, CB, PF, WPE) (const void*)&rag_fit_queue<C, CB, PF, WPE, float, false>

// which, width, waves/EU, unroll (here: surfaces per staged hit chunk), name,
// kernel, learned, fp64, 2D update, one workgroup per block.  Names: c<C>
// surfaces per hit chunk, b<CB> per surface-type/value chunk, pf prefetch,
// e<N> compiled for N waves per SIMD, queue the persistent grid.
void append_ragged_variants(std::vector<Variant>& v) {
    // the first is the default (the fastest measured on the 10^6-track workload)
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_c4b16_pf", RAG_GRID(4, 16, true, 0, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_c4b16", RAG_GRID(4, 16, false, 0, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 4, 4, "rag_fit_c4b16_e4", RAG_GRID(4, 16, false, 4, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_c4b8", RAG_GRID(4, 8, false, 0, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_c4b4", RAG_GRID(4, 4, false, 0, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 0, 8, "rag_fit_c8b16", RAG_GRID(8, 16, false, 0, float, false), false, false, false, true});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_c4b16_queue", RAG_QUEUE(4, 16, false, 0), false, false, false, false});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_f64", RAG_GRID(4, 16, false, 2, double, false), false, true, false, true});
    v.push_back(Variant{2, RAG_W, 4, 4, "rag_fit_2d", RAG_GRID(4, 16, false, 4, float, true), false, false, true, true});
    v.push_back(Variant{2, RAG_W, 0, 4, "rag_fit_f64_2d", RAG_GRID(4, 16, false, 2, double, true), false, true, true, true});
}

// ------------------------------------------------------ autotuner input
// Synthetic ragged tracks: pT in [0.5, 10] GeV, eta in [-2.5, 2.5], phi
// uniform, from the origin; surfaces in crossing order among cylinders at
// r = 2.5 .. 110 cm and disks at |z| = 30 .. 270 cm (25 of each, on the
// track's side in z), the next one being whichever of the next cylinder and
// the next disk the helix reaches first.  Hits are the exact crossings with
// the fit workloads' hit covariance; slots past the point where the track
// leaves the volume (or needs more than half a turn) get a NaN hit, which
// the fit skips (HIT_MISSING).
__global__ void rag_synth(int32_t n, int lmax, const int64_t* offsets, uint8_t* stype, float* sval, float* hpos,
                          float* hcov, float* par, float* cov, int8_t* q) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float pt = 0.5f + 9.5f * hash_u01(t, 1);
    const float eta = -2.5f + 5.0f * hash_u01(t, 2);
    const float phi0 = -PI_F + TWO_PI_F * hash_u01(t, 3);
    const float qq = hash_u01(t, 4) < 0.5f ? -1.0f : 1.0f;
    const float th = 2.0f * atanf(expf(-eta));
    const float p6[6] = {0.0f, 0.0f, 0.0f, 1.0f / pt, phi0, th};
    for (int f = 0; f < 6; ++f) par[(size_t)t * 6 + f] = p6[f];
    for (int k = 0; k < 21; ++k) cov[(size_t)t * 21 + k] = 0.0f;
    cov[(size_t)t * 21 + I21(0, 0)] = 0.01f; cov[(size_t)t * 21 + I21(1, 1)] = 0.01f;
    cov[(size_t)t * 21 + I21(2, 2)] = 1.0f; cov[(size_t)t * 21 + I21(3, 3)] = 1e-4f;
    cov[(size_t)t * 21 + I21(4, 4)] = 1e-4f; cov[(size_t)t * 21 + I21(5, 5)] = 1e-4f;
    q[t] = qq > 0.0f ? 1 : -1;
    const float w = -qq * KAPPA * 3.8f / pt;
    const float cot = cosf(th) / sinf(th);
    const float zs = cot >= 0.0f ? 1.0f : -1.0f;
    float x = 0.0f, y = 0.0f, z = 0.0f, ph = phi0;
    int ic = 0, kd = 0;
    bool alive = true;
    const int64_t h0 = offsets[t], L = offsets[t + 1] - h0;
    for (int64_t j = 0; j < L; ++j) {
        const int64_t h = h0 + j;
        float m[3] = {NAN, NAN, NAN};
        int type = 0;
        float val = 0.0f;
        if (alive && (ic < 25 || kd < 25)) {
            float sphi, cphi;
            sincosf(ph, &sphi, &cphi);
            float sc = INFINITY, sd = INFINITY;
            HelixT<float> hc, hd;
            if (ic < 25) {
                const float R = 2.5f + (float)ic * (107.5f / 24.0f);
                bool lok;
                int it = 0;
                float sn;
                if (cylinder_reachable(x, y, cphi, sphi, w, R) &&
                    newton_cylinder(x, y, cphi, sphi, w, R, newton_tol(1e-6f, R), 16,
                                    line_path(x, y, cphi, sphi, R, &lok), sn, hc, it) &&
                    sn > 0.0f && fabsf(w * sn) <= PI_F)
                    sc = sn;
            }
            if (kd < 25 && cot != 0.0f) {
                const float Z = zs * (30.0f + (float)kd * 10.0f);
                const float sn = (Z - z) / cot;
                if (sn > 0.0f && fabsf(w * sn) <= PI_F) {
                    sd = sn;
                    helix_at(x, y, cphi, sphi, w, sd, hd);
                }
            }
            if (sc < sd) {
                type = 0; val = 2.5f + (float)ic * (107.5f / 24.0f); ++ic;
                x = hc.x; y = hc.y; z = z + sc * cot; ph = ph + 2.0f * hc.u;
            } else if (sd < INFINITY) {
                type = 1; val = zs * (30.0f + (float)kd * 10.0f); ++kd;
                x = hd.x; y = hd.y; z = val; ph = ph + 2.0f * hd.u;
            } else {
                alive = false;
            }
            if (alive && (x * x + y * y > 110.0f * 110.0f * 1.0001f || fabsf(z) > 270.0f * 1.0001f)) alive = false;
            if (alive) { m[0] = x; m[1] = y; m[2] = z; }
        }
        stype[h] = (uint8_t)type;
        sval[h] = val;
        for (int k = 0; k < 3; ++k) hpos[h * 3 + k] = m[k];
        const float V[6] = {1e-4f, 0.0f, 1e-4f, 0.0f, 0.0f, type == 0 ? 1e-2f : 1e-4f};
        for (int k = 0; k < 6; ++k) hcov[h * 6 + k] = V[k];
    }
}

hipError_t launch_ragged_synth(int32_t n, int lmax, const int64_t* offsets, uint8_t* stype, float* sval,
                               float* hpos, float* hcov, float* par, float* cov, int8_t* q, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rag_synth, dim3((n + 255) / 256), dim3(256), 0, s, n, lmax, offsets, stype, sval, hpos, hcov,
                       par, cov, q);
    return hipGetLastError();
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
        hipLaunchKernelGGL(rag_scatter, dim3((unsigned)nwg), dim3(tb), 3 * lds_keys + sizeof(int32_t) * tb, s, aa);
        void* args[] = {&aa, &pp};
        hipError_t e = hipLaunchKernel(v.fn, dim3(v.per_block ? a.nb : a.grid), dim3(RAG_W), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace p2r
