// Load-balancing library: device templates that walk the edges of a set of
// source vertices and hand every edge to an edge functor.
//
// Strategies (GPU Optimization Space section, "Load Balancing"; the Load
// Balancing Library paragraph of the GPU Backend section; the ETWC
// algorithm of the GPU-Specific Optimizations section):
//   VP     one lane per source vertex
//   WM     each wavefront takes 64 consecutive sources and its 64 lanes stride
//          over their concatenated edge lists (owner found by binary search
//          over the wave's degree scan in LDS)
//   CM     the same per workgroup (256 sources, block scan in LDS)
//   STRICT every workgroup takes an equal slice of the frontier's edges
//          (merge path over a device-wide degree scan)
//   TWC    grid-wide binning by degree into lane / wave / workgroup tiers,
//          each tier processed by its own pass
//   ETWC   per workgroup: each lane splits its vertex's edges into a
//          workgroup-multiple chunk, a 64-multiple chunk and a remainder,
//          queued in LDS and processed by the workgroup, a wave and a lane
//
// Every strategy is a __device__ function with a grid-stride outer loop, so
// the same code runs as its own kernel and inside a fused persistent kernel.
//
// Edge functor F:
//   bool active(x)          -- process x's edges at all
//   int  edge(x, y, e)      -- process edge e = (x, y); returns the vertex to
//                              put in the output frontier, or -1
//   bool done(x)            -- stop scanning x's edges early (pull)
//   Pre load(x, y, e)       -- the edge's reads, no side effects (batched
//   int apply(x, y, e, pre)    loops issue a batch's loads, then its applies)
//   Tok issue(x, y, e, pre, ok), int finish(x, y, e, pre, ok, tok)
//                           -- optional two-phase apply (see TwoPhase below)
//   begin(), flush()        -- workgroup-uniform hooks around staged work
#pragma once

#include <type_traits>

#include "common.hpp"
#include "frontier.hpp"

namespace gg {

// Functors whose update is one atomic may split apply() in two: issue(..., ok)
// makes the atomic (when ok and the filter passes) and returns its raw result
// as a Tok, finish(..., ok, tok) turns that into apply()'s return value. A
// batch then issues all its atomics before reading any result: with apply()
// the result is compared inside the branch that guards the atomic, so the
// compiler waits for each atomic before issuing the next.
template <class F, class = void>
struct TwoPhase : std::false_type {};
template <class F>
struct TwoPhase<F, std::void_t<typename F::Tok>> : std::true_type {};

// the updates of a batch of B edges (uu[b], vv[b], ee[b]) with their loaded
// values pp[b]; ok[b] false skips an edge. xx[b] gets apply()'s result or -1.
template <int B, class F>
__device__ __forceinline__ void apply_batch(F &f, const int *uu, const int *vv, const int *ee,
                                            const typename F::Pre *pp, const bool *ok, int *xx, long long &ne) {
    if constexpr (TwoPhase<F>::value) {
        typename F::Tok tk[B];
        bool go[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            go[b] = ok[b] && !f.done(uu[b]);
            tk[b] = f.issue(uu[b], vv[b], ee[b], pp[b], go[b]);
        }
#pragma unroll
        for (int b = 0; b < B; b++) {
            xx[b] = f.finish(uu[b], vv[b], ee[b], pp[b], go[b], tk[b]);
            ne += go[b];
        }
    } else {
#pragma unroll
        for (int b = 0; b < B; b++) {
            xx[b] = -1;
            if (ok[b] && !f.done(uu[b])) {
                xx[b] = f.apply(uu[b], vv[b], ee[b], pp[b]);
                ne++;
            }
        }
    }
}

// Edges a lane loads before applying them (load-balancer loops that issue
// each edge's column and functor reads for several edges at once, so their
// latencies overlap instead of adding up)
constexpr int kEdgeBatch = 4;

struct Tid {  // position of this lane in the (possibly persistent) grid
    int block, nblocks;
    __device__ static Tid here() { return Tid{(int)blockIdx.x, (int)gridDim.x}; }
};

// ---------------------------------------------------------------------------- VP
// One lane per frontier vertex walks its edges a batch at a time: the
// batch's column reads, then its functor reads, then its updates are each
// issued back to back, so a hub's serial walk pays three memory round trips
// per batch. Appends are staged per workgroup unless STAGE is false (see
// lb_cm); the staged form takes larger batches when the functor
// loads one word per edge (a hub's walk is the launch's critical path); the
// unstaged one runs inside persistent kernels, where registers bound the
// resident grid.
constexpr int kVpBatch = 16;
constexpr int kVpBatchStaged = 32;
template <int CREATE, int DEDUP, bool STAGE = true, class Src, class F>
__device__ void lb_vp(const DevGraph &g, const Src &src, F &f, const OutFrontier &out, Tid t,
                      long long &ne) {
    __shared__ StageLDS s_st;
    if constexpr (STAGE) {
        if (threadIdx.x == 0) s_st.c = 0;
        f.begin();
        __syncthreads();
    }
    const int stride = t.nblocks * kBlock;
    for (int base = t.block * kBlock; base < src.size; base += stride) {
        const int i = base + (int)threadIdx.x;
        const int u = i < src.size ? src.get(i) : 0;
        int e0 = 0, end = 0;
        if (i < src.size && f.active(u)) {
            e0 = g.row_ptr[u];
            end = g.row_ptr[u + 1];
        }
        // the wavefront takes batches until its longest row is done, every
        // lane in every batch (lanes out of edges apply nothing), so a batch's
        // appends are placed with one scan over the wavefront
        constexpr int B = STAGE && sizeof(typename F::Pre) <= 4 ? kVpBatchStaged : kVpBatch;
        for (;;) {
            const bool has = e0 < end && !f.done(u);
            if (__ballot(has) == 0) break;
            int vv[B], xx[B], uu[B], ee[B];
            typename F::Pre pp[B];
            bool ok[B];
#pragma unroll
            for (int b = 0; b < B; b++) {
                vv[b] = 0;
                pp[b] = typename F::Pre{};
                uu[b] = u;
                ee[b] = e0 + b;
                ok[b] = has && e0 + b < end;
            }
            if (has) {
#pragma unroll
                for (int b = 0; b < B; b++) vv[b] = g.col[e0 + b < end ? e0 + b : end - 1];
#pragma unroll
                for (int b = 0; b < B; b++) pp[b] = f.load(u, vv[b], e0 + b < end ? e0 + b : end - 1);
            }
            apply_batch<B>(f, uu, vv, ee, pp, ok, xx, ne);
            if constexpr (STAGE) {
                emit_staged_batch<CREATE, DEDUP, B>(out, s_st, xx);
            } else {
#pragma unroll
                for (int b = 0; b < B; b++) emit<CREATE, DEDUP>(out, xx[b] >= 0, xx[b]);
            }
            if (has) e0 += B;
        }
        if constexpr (STAGE) {
            emit_flush_half<CREATE>(out, s_st);
            f.flush();
        }
    }
    if constexpr (STAGE) emit_flush<CREATE>(out, s_st);
}

// owner of edge rank j: the last k in [0, len) with scan[k] <= j
__device__ __forceinline__ int owner_search(const int *scan, int len, int j) {
    int lo = 0, hi = len;  // invariant: scan[lo] <= j, answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (scan[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------- WM
template <int CREATE, int DEDUP, class Src, class F>
__device__ void lb_wm(const DevGraph &g, const Src &src, F &f, const OutFrontier &out, Tid t,
                      long long &ne) {
    __shared__ int s_u[kBlock], s_beg[kBlock], s_scan[kBlock];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    int *wu = s_u + wib * kWave, *wbeg = s_beg + wib * kWave, *wscan = s_scan + wib * kWave;
    const int waves_per_block = kBlock / kWave;
    const int total_waves = t.nblocks * waves_per_block;
    for (int base = (t.block * waves_per_block + wib) * kWave; base < src.size; base += total_waves * kWave) {
        const int i = base + lane;
        int u = 0, deg = 0, beg = 0;
        if (i < src.size) {
            u = src.get(i);
            if (f.active(u)) { beg = g.row_ptr[u]; deg = g.row_ptr[u + 1] - beg; }
        }
        const int incl = wave_incl_scan(deg);
        const int total = wave_bcast(incl, kWave - 1);
        wu[lane] = u; wbeg[lane] = beg; wscan[lane] = incl - deg;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int j = lane; j < total; j += kWave) {
            const int k = owner_search(wscan, kWave, j);
            const int uu = wu[k];
            if (f.done(uu)) continue;
            const int e = wbeg[k] + (j - wscan[k]);
            const int x = f.edge(uu, g.col[e], e);
            emit<CREATE, DEDUP>(out, x >= 0, x);
            ne++;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// block-wide exclusive scan of one int per thread; returns the block total
__device__ __forceinline__ int block_excl_scan(int x, int &excl, int *s_tmp /* kBlock/kWave */) {
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    const int incl = wave_incl_scan(x);
    if (lane == kWave - 1) s_tmp[wib] = incl;
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) {
        const int v = s_tmp[w];
        if (w < wib) off += v;
        total += v;
    }
    excl = off + incl - x;
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------- CM
// STAGE: appends staged per workgroup (the default); the persistent kernels
// on high-diameter graphs, whose few workgroups rarely contend, append per
// wavefront instead and skip the flush barriers
template <int CREATE, int DEDUP, bool STAGE = true, class Src, class F>
__device__ void lb_cm(const DevGraph &g, const Src &src, F &f, const OutFrontier &out, Tid t,
                      long long &ne) {
    __shared__ int s_u[kBlock], s_beg[kBlock], s_scan[kBlock], s_tmp[kBlock / kWave];
    __shared__ StageLDS s_st;
    if (threadIdx.x == 0) s_st.c = 0;
    if constexpr (STAGE) f.begin();
    __syncthreads();
    for (int base = t.block * kBlock; base < src.size; base += t.nblocks * kBlock) {
        const int i = base + (int)threadIdx.x;
        int u = 0, deg = 0, beg = 0;
        if (i < src.size) {
            u = src.get(i);
            if (f.active(u)) { beg = g.row_ptr[u]; deg = g.row_ptr[u + 1] - beg; }
        }
        int excl;
        const int total = block_excl_scan(deg, excl, s_tmp);
        s_u[threadIdx.x] = u; s_beg[threadIdx.x] = beg; s_scan[threadIdx.x] = excl;
        __syncthreads();
        for (int j = threadIdx.x; j < total; j += kBlock) {
            const int k = owner_search(s_scan, kBlock, j);
            const int uu = s_u[k];
            if (f.done(uu)) continue;
            const int e = s_beg[k] + (j - s_scan[k]);
            const int x = f.edge(uu, g.col[e], e);
            if constexpr (STAGE) emit_staged<CREATE, DEDUP>(out, s_st, x >= 0, x);
            else emit<CREATE, DEDUP>(out, x >= 0, x);
            ne++;
        }
        __syncthreads();
        if constexpr (STAGE) {
            emit_flush_half<CREATE>(out, s_st);
            f.flush();
        }
    }
    if constexpr (STAGE) emit_flush<CREATE>(out, s_st);
}

// ---------------------------------------------------------------------------- ETWC
template <int CREATE, int DEDUP, bool STAGE = true, class Src, class F>
__device__ void lb_etwc(const DevGraph &g, const Src &src, F &f, const OutFrontier &out, Tid t,
                        long long &ne) {
    // Q[0] lane stage, Q[1] wave stage, Q[2] workgroup stage: {begin, end, vertex}
    __shared__ int q_beg[3][kBlock], q_end[3][kBlock], q_u[3][kBlock];
    __shared__ int q_n[3];
    __shared__ StageLDS s_st;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    if (tid == 0) s_st.c = 0;
    if constexpr (STAGE) f.begin();
    __syncthreads();
    for (int base = t.block * kBlock; base < src.size; base += t.nblocks * kBlock) {
        if (tid < 3) q_n[tid] = 0;
        __syncthreads();
        const int i = base + tid;
        if (i < src.size) {
            const int u = src.get(i);
            if (f.active(u)) {
                int beg = g.row_ptr[u];
                const int end = g.row_ptr[u + 1];
                int size = end - beg;
                const int s2 = (size / kBlock) * kBlock;
                if (s2 > 0) {
                    const int k = atomicAdd(&q_n[2], 1);
                    q_beg[2][k] = beg; q_end[2][k] = beg + s2; q_u[2][k] = u;
                    beg += s2; size -= s2;
                }
                const int s1 = (size / kWave) * kWave;
                if (s1 > 0) {
                    const int k = atomicAdd(&q_n[1], 1);
                    q_beg[1][k] = beg; q_end[1][k] = beg + s1; q_u[1][k] = u;
                    beg += s1; size -= s1;
                }
                if (size > 0) {
                    const int k = atomicAdd(&q_n[0], 1);
                    q_beg[0][k] = beg; q_end[0][k] = end; q_u[0][k] = u;
                }
            }
        }
        __syncthreads();
        // stage 0: one lane per entry, its edges in batches of kEdgeBatch
        for (int k = tid; k < q_n[0]; k += kBlock) {
            const int u = q_u[0][k], end = q_end[0][k];
            for (int e0 = q_beg[0][k]; e0 < end; e0 += kEdgeBatch) {
                int vv[kEdgeBatch];
                typename F::Pre pp[kEdgeBatch];
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) vv[b] = g.col[e0 + b < end ? e0 + b : end - 1];
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) pp[b] = f.load(u, vv[b], e0 + b < end ? e0 + b : end - 1);
                int xx[kEdgeBatch], uu[kEdgeBatch], ee[kEdgeBatch];
                bool ok[kEdgeBatch];
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) {
                    uu[b] = u;
                    ee[b] = e0 + b;
                    ok[b] = e0 + b < end;
                }
                apply_batch<kEdgeBatch>(f, uu, vv, ee, pp, ok, xx, ne);
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) {
                    if constexpr (STAGE) emit_staged<CREATE, DEDUP>(out, s_st, xx[b] >= 0, xx[b]);
                    else emit<CREATE, DEDUP>(out, xx[b] >= 0, xx[b]);
                }
            }
        }
        // stage 1: one wavefront per entry, lanes cyclic over its edges
        for (int k = wib; k < q_n[1]; k += kBlock / kWave) {
            const int u = q_u[1][k], end = q_end[1][k];
            for (int e = q_beg[1][k] + lane; e < end; e += kWave) {
                if (f.done(u)) break;
                const int x = f.edge(u, g.col[e], e);
                if constexpr (STAGE) emit_staged<CREATE, DEDUP>(out, s_st, x >= 0, x);
                else emit<CREATE, DEDUP>(out, x >= 0, x);
                ne++;
            }
        }
        // stage 2: the whole workgroup per entry
        for (int k = 0; k < q_n[2]; k++) {
            const int u = q_u[2][k], end = q_end[2][k];
            for (int e = q_beg[2][k] + tid; e < end; e += kBlock) {
                if (f.done(u)) break;
                const int x = f.edge(u, g.col[e], e);
                if constexpr (STAGE) emit_staged<CREATE, DEDUP>(out, s_st, x >= 0, x);
                else emit<CREATE, DEDUP>(out, x >= 0, x);
                ne++;
            }
        }
        __syncthreads();
        if constexpr (STAGE) {
            emit_flush_half<CREATE>(out, s_st);
            f.flush();
        }
    }
    if constexpr (STAGE) emit_flush<CREATE>(out, s_st);
}

// ---------------------------------------------------------------------------- TWC
// Tier thresholds: degree >= kBlock -> workgroup tier, >= kWave -> wave tier,
// else lane tier.
struct TwcBins {
    int32_t *q[3];
    int32_t *count;  // [3]
    int32_t cap;
    int32_t *overflow;
};

template <class Src, class F>
__device__ void twc_bin(const DevGraph &g, const Src &src, F &f, const TwcBins &b, Tid t) {
    const int stride = t.nblocks * kBlock;
    const int n_iter = (src.size + stride - 1) / stride;
    for (int it = 0; it < n_iter; it++) {  // wave-uniform trip count for the ballots
        const int i = it * stride + t.block * kBlock + (int)threadIdx.x;
        int u = -1, tier = -1;
        if (i < src.size) {
            u = src.get(i);
            if (f.active(u)) {
                const int d = g.row_ptr[u + 1] - g.row_ptr[u];
                tier = d >= kBlock ? 2 : (d >= kWave ? 1 : (d > 0 ? 0 : -1));
            }
        }
#pragma unroll
        for (int k = 0; k < 3; k++) wave_append(b.q[k], b.count + k, b.cap, b.overflow, tier == k, u);
    }
}

struct SrcQueueDev {  // queue whose size lives in device memory
    const int32_t *ids;
    const int32_t *size_ptr;
};

// tier 1: one wavefront per vertex
template <int CREATE, int DEDUP, class F>
__device__ void twc_wave_tier(const DevGraph &g, const int32_t *ids, int size, F &f, const OutFrontier &out,
                              Tid t, long long &ne) {
    const int lane = lane_id();
    const int wpb = kBlock / kWave;
    for (int k = t.block * wpb + (int)threadIdx.x / kWave; k < size; k += t.nblocks * wpb) {
        const int u = ids[k];
        const int end = g.row_ptr[u + 1];
        for (int e = g.row_ptr[u] + lane; e < end; e += kWave) {
            if (f.done(u)) break;
            const int x = f.edge(u, g.col[e], e);
            emit<CREATE, DEDUP>(out, x >= 0, x);
            ne++;
        }
    }
}

// tier 2: one workgroup per vertex
template <int CREATE, int DEDUP, class F>
__device__ void twc_block_tier(const DevGraph &g, const int32_t *ids, int size, F &f,
                               const OutFrontier &out, Tid t, long long &ne) {
    for (int k = t.block; k < size; k += t.nblocks) {
        const int u = ids[k];
        const int end = g.row_ptr[u + 1];
        for (int e = g.row_ptr[u] + (int)threadIdx.x; e < end; e += kBlock) {
            if (f.done(u)) break;
            const int x = f.edge(u, g.col[e], e);
            emit<CREATE, DEDUP>(out, x >= 0, x);
            ne++;
        }
    }
}

// ---------------------------------------------------------------------------- STRICT
// scan[i] = exclusive prefix sum of the degrees of the (active) sources,
// scan[size] = total edges. Each workgroup takes kStrictChunk consecutive
// edge ranks; owners are found by binary search over a window of the scan
// staged in LDS (windows advance when a chunk spans many sources).
constexpr int kStrictChunk = kBlock * 8;

__device__ __forceinline__ int upper_bound_ll(const long long *a, int n, long long x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Last index i in [0, n) with a[i] <= x (a ascending, a[0] <= x), found by a
// whole wavefront: each round the 64 lanes probe 64 evenly spaced positions
// and a ballot keeps the last one that qualifies (log_64 n dependent loads).
__device__ __forceinline__ int wave_last_le(const long long *a, int n, long long x) {
    const int lane = lane_id();
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int step = (hi - lo + kWave - 1) / kWave;
        const int p = lo + lane * step;
        const bool ok = p < hi && a[p] <= x;
        const uint64_t m = __ballot(ok);
        const int hl = 63 - __builtin_clzll(m);
        const int nlo = lo + hl * step;
        hi = min(hi, nlo + step);
        lo = nlo;
    }
    return lo;
}

template <int CREATE, int DEDUP, class Src, class F>
__device__ void lb_strict(const DevGraph &g, const Src &src, const long long *scan, F &f,
                          const OutFrontier &out, Tid t, long long &ne) {
    constexpr int W = kStrictChunk;
    __shared__ long long s_scan[W + 1];
    __shared__ int s_k0, s_k1;
    // FUSED creation stages the window's appends in LDS (one global atomic per
    // window instead of one per wavefront and edge batch)
    __shared__ StageLDS s_st;
    if (threadIdx.x == 0) s_st.c = 0;
    f.begin();
    __syncthreads();
    const long long total = scan[src.size];
    const long long nchunks = (total + W - 1) / W;
    for (long long c = t.block; c < nchunks; c += t.nblocks) {
        const long long r0 = c * W, r1 = (r0 + W < total) ? r0 + W : total;
        // owners of r0 and r1-1 (waves 0 and 1 search in parallel)
        if (threadIdx.x < kWave) {
            const int k = wave_last_le(scan, src.size + 1, r0);
            if (threadIdx.x == 0) s_k0 = k;
        } else if (threadIdx.x < 2 * kWave) {
            const int k = wave_last_le(scan, src.size + 1, r1 - 1);
            if (threadIdx.x == kWave) s_k1 = k;
        }
        __syncthreads();
        const int k0 = s_k0, k1 = s_k1;
        __syncthreads();
        for (int kw = k0; kw <= k1; kw += W) {  // LDS windows of sources [kw, kw+W)
            const int wlen = (k1 - kw + 1 < W) ? k1 - kw + 1 : W;
            for (int j = threadIdx.x; j <= wlen; j += kBlock) s_scan[j] = scan[kw + j];
            __syncthreads();
            long long lo = s_scan[0] > r0 ? s_scan[0] : r0;
            long long hi = s_scan[wlen] < r1 ? s_scan[wlen] : r1;
            int a = 0;  // owners only move forward as r grows
            // a lane's ranks r, r + kBlock, ... in batches of kEdgeBatch: owners
            // from LDS, then every batch member's source, row start, column and
            // functor reads are issued before any update (ranks past hi repeat
            // the last valid rank and are not applied)
            for (long long rb = lo + threadIdx.x; rb < hi; rb += (long long)kEdgeBatch * kBlock) {
                int ab[kEdgeBatch], uu[kEdgeBatch], ee[kEdgeBatch], vv[kEdgeBatch];
                typename F::Pre pp[kEdgeBatch];
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) {
                    long long r = rb + (long long)k * kBlock;
                    if (r >= hi) r = hi - 1;
                    int b = wlen;  // last j with s_scan[j] <= r
                    while (b - a > 1) {
                        const int mid = (a + b) >> 1;
                        if (s_scan[mid] <= r) a = mid; else b = mid;
                    }
                    ab[k] = a;
                    ee[k] = (int)(r - s_scan[a]);
                }
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) uu[k] = src.get(kw + ab[k]);
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) ee[k] += g.row_ptr[uu[k]];
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) vv[k] = g.col[ee[k]];
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) pp[k] = f.load(uu[k], vv[k], ee[k]);
                int xx[kEdgeBatch];
                bool ok[kEdgeBatch];
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) ok[k] = rb + (long long)k * kBlock < hi;
                apply_batch<kEdgeBatch>(f, uu, vv, ee, pp, ok, xx, ne);
#pragma unroll
                for (int k = 0; k < kEdgeBatch; k++) emit_staged<CREATE, DEDUP>(out, s_st, xx[k] >= 0, xx[k]);
            }
            __syncthreads();
            emit_flush_half<CREATE>(out, s_st);
            f.flush();
        }
    }
    emit_flush<CREATE>(out, s_st);
}

// ---------------------------------------------------------------------------- EDGE_ONLY
// Edge-parallel over all CSR entries; a source participates when it is in the
// input frontier's boolmap (null map = every vertex).
template <int CREATE, int DEDUP, class F>
__device__ void lb_edge_only(const DevGraph &g, const uint8_t *member, F &f, const OutFrontier &out, Tid t,
                             long long &ne) {
    const long long stride = (long long)t.nblocks * kBlock;
    for (long long e = (long long)t.block * kBlock + threadIdx.x; e < g.m; e += stride) {
        const int u = g.coo_src[e];
        bool take = member == nullptr || member[u];
        take = take && f.active(u) && !f.done(u);
        int x = -1;
        if (take) { x = f.edge(u, g.col[e], (int)e); ne++; }
        emit<CREATE, DEDUP>(out, x >= 0, x);
    }
}

// per-wave reduction of the examined-edge counter
__device__ __forceinline__ void flush_edge_count(long long ne, unsigned long long *counter) {
    if (counter == nullptr) return;
    const long long s = wave_sum(ne);
    if (lane_id() == 0 && s) atomic_add_u64(counter, (unsigned long long)s);
}

}  // namespace gg
