// Batched multi-source SSSP: up to 64 delta-stepping queries on one graph run
// in one persistent launch that walks a single, shared bucket sequence.
//
// Delta-stepping (the applyUpdatePriority operator with configDelta) settles
// bucket k = [k*delta, (k+1)*delta) before any later bucket. Sharing the
// bucket index across sources keeps that order per source: bucket k is
// processed for every source that has entries in it and skipped by the
// others, exactly as a lone query skips its empty buckets. Distances are
// unique, so every source's result equals the single-source answer bit for
// bit; what the batch shares is the grid barrier of each round, which is the
// cost that dominates high-diameter graphs (Kernel Fusion across Iterations).
//
// State per vertex v: dist[v*K + j] (vertex-major), a near-set word per
// round parity (bit j: source j must relax v's edges in the next round) and
// a far-set word (bit j: dist_j(v) lies beyond the current bucket). A vertex
// enters a queue when its word goes from zero to non-zero, so each queue
// holds a vertex at most once. A round reads the near words of its queue
// (and clears them), and relaxes every (edge, source) pair: an improved
// distance still inside the bucket sets the next round's near bit, a later
// one the far bit. When a round produces no near entries, the next bucket is
// the smallest floor(dist/delta) over far bits beyond the current bucket;
// those bits move to the near set, later ones stay, and bits whose distance
// fell back into a settled bucket are dropped.
//
// With unit weights and an unbounded bucket every improvement joins the next
// round, so a round is one BFS level: the same loop is the PUSH form of the
// batched BFS (one barrier per level, work proportional to the frontier),
// which suits high-diameter graphs where the bit-packed PULL sweep would
// scan every vertex once per level.
//
// Work in a round is spread like CM (one workgroup per kMsBlock queue
// entries): an exclusive scan of popcount(word) * degree gives every (edge,
// source) pair a rank, lanes stride over the ranks, and the sources of one
// edge sit on neighbouring lanes, so their distance words share cache lines.
// The loop is bound by the latency of its dependent accesses (entry, row
// range, column, distance, atomic, append), so it runs few, wide workgroups:
// many waves in flight per compute unit while the grid barrier, whose cost
// grows with the number of workgroups, stays cheap.
#include <climits>

#include "algos.hpp"
#include "driver.hpp"
#include "fused.hpp"
#include "ms.hpp"

namespace gg {

using u64 = unsigned long long;

constexpr int kMsBlock = 1024;  // lanes per workgroup of the batched loop

// index of the i-th set bit of m (i < popcount(m)), by halving the window
__device__ __forceinline__ int select_bit(u64 m, int i) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll(m & ((1ull << w) - 1ull));
        if (i >= c) { i -= c; m >>= w; pos += w; }
    }
    return pos;
}

// block-wide exclusive scan of one 64-bit value per thread; returns the total
__device__ __forceinline__ long long block_excl_scan64(long long x, long long &excl, long long *s_tmp) {
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    const long long incl = wave_incl_scan64(x);
    if (lane == kWave - 1) s_tmp[wib] = incl;
    __syncthreads();
    long long off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kMsBlock / kWave; w++) {
        const long long v = s_tmp[w];
        if (w < wib) off += v;
        total += v;
    }
    excl = off + incl - x;
    __syncthreads();
    return total;
}

__device__ __forceinline__ int last_le64(const long long *a, int n, long long x) {
    int lo = 0, hi = n;  // a[lo] <= x
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ctr: [0..2] near sizes (rotating by round), [3..4] far sizes (by far epoch),
// [5..6] bucket minima (by advance), [8] rounds, [9] buckets, [10] an
// unrepresentable distance was seen, [12] queue overflow
struct MsSsspArgs {
    DevGraph g;
    int K;
    int32_t *dist;
    u64 *near0, *near1, *far;
    int32_t *q0, *q1, *farq0, *farq1;
    int32_t *ctr;
    int32_t delta;
    GridBarrier bar;
};

__global__ __launch_bounds__(kBlock) void k_mssssp_init(int n, int K, const int32_t *srcs, int32_t *dist,
                                                        u64 *near0, u64 *near1, u64 *far, int32_t *q0,
                                                        int32_t *count, int32_t *overflow) {
    __shared__ int s_src[64];
    if (threadIdx.x < 64) s_src[threadIdx.x] = (int)threadIdx.x < K ? srcs[threadIdx.x] : -1;
    __syncthreads();
    const int n_iter = (n + gridDim.x * kBlock - 1) / (gridDim.x * kBlock);
    for (int it = 0; it < n_iter; it++) {
        const int v = (it * gridDim.x + blockIdx.x) * kBlock + threadIdx.x;
        u64 mask = 0;
        if (v < n) {
            for (int j = 0; j < K; j++) {
                const bool on = s_src[j] == v;
                if (on) mask |= 1ull << j;
                dist[(size_t)v * K + j] = on ? 0 : INT_MAX;
            }
            near0[v] = mask;
            near1[v] = 0;
            far[v] = 0;
        }
        wave_append(q0, count, n, overflow, mask != 0, v);
    }
}

// relax one (edge, source) pair; every active lane of the wave calls the
// appends together
template <bool UNIT>
__device__ __forceinline__ void ms_relax_pair(const MsSsspArgs &a, int du, int e, int v, int src, u64 *nnext,
                                              const Staged &nq, const Staged &fq, long long bucket_end) {
    const long long nd = (long long)du + (UNIT ? 1ll : (long long)a.g.w[e]);
    int32_t *dv = &a.dist[(size_t)v * a.K + src];
    bool to_near = false, to_far = false;
    if (nd > (long long)INT_MAX - 1) {
        if (*dv == INT_MAX) a.ctr[10] = 1;  // confirmed after the loop
    } else if (nd < *dv) {
        const int old = atomic_min_i32(dv, (int)nd);
        if (nd < old) {
            const u64 bit = 1ull << src;
            if (nd < bucket_end) to_near = atomic_or_u64(&nnext[v], bit) == 0;
            else to_far = atomic_or_u64(&a.far[v], bit) == 0;
        }
    }
    stage_append(nq, a.g.n, a.ctr + 12, to_near, v);
    stage_append(fq, a.g.n, a.ctr + 12, to_far, v);
}

// In a full round (a workgroup's share of the queue is at least kMsBlock
// entries) entries with at most kMsLaneWork (edge, source) pairs are relaxed
// by their own lane and larger ones are spread over the workgroup by rank. A
// smaller round is divided evenly over all workgroups and every entry's pairs
// are spread by rank, so that each lane holds about one pair: such rounds are
// bound by the latency of one relaxation, not by throughput.
constexpr int kMsLaneWork = 32;

// one round: relax the (edge, source) pairs of the near queue
template <bool UNIT>
__device__ __forceinline__ void ms_relax(const MsSsspArgs &a, const int32_t *qin, int cnt, u64 *ncur, u64 *nnext,
                                         int32_t *qout, int32_t *qcount, int32_t *farq, int32_t *farc,
                                         long long bucket_end, Tid t) {
    __shared__ long long s_scan[kMsBlock + 1], s_tmp[kMsBlock / kWave];
    __shared__ int s_u[kMsBlock], s_beg[kMsBlock], s_p[kMsBlock];
    __shared__ u64 s_m[kMsBlock];
    __shared__ int32_t s_nq[kStage], s_fq[kStage];
    __shared__ int s_nc, s_fc, s_base;
    if (threadIdx.x == 0) { s_nc = 0; s_fc = 0; }
    __syncthreads();
    const Staged nq{s_nq, &s_nc, qout, qcount}, fq{s_fq, &s_fc, farq, farc};
    const int K = a.K;
    const int share = (cnt + t.nblocks - 1) / t.nblocks;
    const int chunk = share < kMsBlock ? share : kMsBlock;  // entries per workgroup step (uniform)
    const bool full = chunk == kMsBlock;
    for (int base = t.block * chunk; base < cnt; base += t.nblocks * chunk) {
        const int i = base + (int)threadIdx.x;
        int u = 0, beg = 0, end = 0, p = 0;
        u64 m = 0;
        long long work = 0;
        if ((int)threadIdx.x < chunk && i < cnt) {
            u = qin[i];
            m = ncur[u];
            ncur[u] = 0;  // only this entry reads or clears it in this round
            p = __popcll(m);
            beg = a.g.row_ptr[u];
            end = a.g.row_ptr[u + 1];
            work = (long long)p * (end - beg);
        }
        const bool own = full && work <= kMsLaneWork;
        // small entries: this lane walks its edges, and per edge its sources
        if (own) {
            for (int e = beg; e < end; e++) {
                const int v = a.g.col[e];
                u64 mm = m;
                while (mm) {
                    const int src = __ffsll(mm) - 1;
                    mm &= mm - 1;
                    ms_relax_pair<UNIT>(a, a.dist[(size_t)u * K + src], e, v, src, nnext, nq, fq, bucket_end);
                }
            }
        }
        // large entries: ranks over the workgroup, sources of an edge on adjacent lanes
        long long excl;
        const long long total = block_excl_scan64(own ? 0 : work, excl, s_tmp);
        if (total > 0) {  // uniform: every lane read the same total
            s_u[threadIdx.x] = u; s_beg[threadIdx.x] = beg; s_p[threadIdx.x] = p; s_m[threadIdx.x] = m;
            s_scan[threadIdx.x] = excl;
            __syncthreads();
            for (long long j = threadIdx.x; j < total; j += kMsBlock) {
                const int o = last_le64(s_scan, chunk, j);
                const unsigned r = (unsigned)(j - s_scan[o]);
                const unsigned po = (unsigned)s_p[o];
                const unsigned el = r / po;
                const int src = select_bit(s_m[o], (int)(r - el * po));
                const int e = s_beg[o] + (int)el;
                ms_relax_pair<UNIT>(a, a.dist[(size_t)s_u[o] * K + src], e, a.g.col[e], src, nnext, nq, fq,
                                    bucket_end);
            }
        }
        stage_flush(nq, a.g.n, a.ctr + 12, &s_base);
        stage_flush(fq, a.g.n, a.ctr + 12, &s_base);
    }
}

// smallest bucket index beyond k over the far bits
__device__ __forceinline__ void ms_far_min(const MsSsspArgs &a, const int32_t *farq, int fc, int k, int32_t *kmin,
                                           Tid t) {
    int local = INT_MAX;
    for (int i = t.block * kMsBlock + (int)threadIdx.x; i < fc; i += t.nblocks * kMsBlock) {
        const int v = farq[i];
        u64 m = a.far[v];
        while (m) {
            const int j = __ffsll(m) - 1;
            m &= m - 1;
            const int b = a.dist[(size_t)v * a.K + j] / a.delta;
            if (b > k && b < local) local = b;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int o = __shfl_xor(local, off, kWave);
        local = o < local ? o : local;
    }
    if (lane_id() == 0 && local != INT_MAX && local < load_relaxed(kmin)) atomic_min_i32(kmin, local);
}

// far bits of bucket knew -> near set; later buckets stay; settled ones are dropped
__device__ __forceinline__ void ms_far_split(const MsSsspArgs &a, const int32_t *farq, int fc, int knew,
                                             u64 *nnext, int32_t *qout, int32_t *qcount, int32_t *nfarq,
                                             int32_t *nfarc, Tid t) {
    __shared__ int32_t s_nq[kStage], s_fq[kStage];
    __shared__ int s_nc, s_fc, s_base;
    if (threadIdx.x == 0) { s_nc = 0; s_fc = 0; }
    __syncthreads();
    const Staged nq{s_nq, &s_nc, qout, qcount}, fq{s_fq, &s_fc, nfarq, nfarc};
    const int stride = t.nblocks * kMsBlock;
    const int n_iter = (fc + stride - 1) / stride;
    for (int it = 0; it < n_iter; it++) {
        const int i = it * stride + t.block * kMsBlock + (int)threadIdx.x;
        u64 move = 0, keep = 0;
        int v = 0;
        if (i < fc) {
            v = farq[i];
            u64 m = a.far[v];
            while (m) {
                const int j = __ffsll(m) - 1;
                m &= m - 1;
                const int b = a.dist[(size_t)v * a.K + j] / a.delta;
                if (b == knew) move |= 1ull << j;
                else if (b > knew) keep |= 1ull << j;
            }
            a.far[v] = keep;
            if (move) nnext[v] = move;  // the near set is empty when a bucket advances
        }
        stage_append(nq, a.g.n, a.ctr + 12, move != 0, v);
        stage_append(fq, a.g.n, a.ctr + 12, keep != 0, v);
        stage_flush(nq, a.g.n, a.ctr + 12, &s_base);
        stage_flush(fq, a.g.n, a.ctr + 12, &s_base);
    }
}

template <bool UNIT>
__global__ __launch_bounds__(kMsBlock) void k_mssssp_fused(MsSsspArgs a) {
    const Tid t = Tid::here();
    GridBarrier bar = a.bar;
    int r = 0, k = 0, fe = 0, adv = 0, rounds = 0;
    const bool lead = t.block == 0 && threadIdx.x == 0;
    for (;;) {
        // queue sizes are at most n (a vertex enters a queue once); the clamps
        // keep reads in bounds even if a count ever ran past the capacity
        const int cnt = min(load_relaxed(&a.ctr[r % 3]), a.g.n);
        if (lead) __hip_atomic_store(&a.ctr[(r + 2) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t *qin = (r & 1) ? a.q1 : a.q0;
        int32_t *qout = (r & 1) ? a.q0 : a.q1;
        u64 *ncur = (r & 1) ? a.near1 : a.near0;
        u64 *nnext = (r & 1) ? a.near0 : a.near1;
        int32_t *qcount = &a.ctr[(r + 1) % 3];
        int32_t *farq = (fe & 1) ? a.farq1 : a.farq0;
        int32_t *farc = a.ctr + 3 + (fe & 1);
        if (cnt > 0) {
            const long long bucket_end = UNIT ? LLONG_MAX : (long long)(k + 1) * a.delta;
            ms_relax<UNIT>(a, qin, cnt, ncur, nnext, qout, qcount, farq, farc, bucket_end, t);
            rounds++;
        } else {
            const int fc = min(load_relaxed(farc), a.g.n);
            if (fc == 0) break;
            int32_t *kmin = a.ctr + 5 + (adv & 1);
            if (lead) {
                __hip_atomic_store(a.ctr + 5 + ((adv + 1) & 1), INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(a.ctr + 3 + ((fe + 1) & 1), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ms_far_min(a, farq, fc, k, kmin, t);
            if (!grid_sync(bar)) break;
            const int knew = load_relaxed(kmin);
            if (knew == INT_MAX) break;
            int32_t *nfarq = (fe & 1) ? a.farq0 : a.farq1;
            ms_far_split(a, farq, fc, knew, nnext, qout, qcount, nfarq, a.ctr + 3 + ((fe + 1) & 1), t);
            fe++;
            adv++;
            k = knew;
        }
        if (!grid_sync(bar)) break;
        r++;
    }
    if (lead) { a.ctr[8] = rounds; a.ctr[9] = adv + 1; }
}

// After the loop: source j overflowed when some vertex it did not reach has a
// neighbour it did reach (every relaxation into it was unrepresentable).
__global__ __launch_bounds__(kBlock) void k_mssssp_overflow_check(DevGraph g, int K, const int32_t *dist,
                                                                  u64 *bad) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < g.n; v += gridDim.x * kBlock) {
        u64 unreached = 0;
        for (int j = 0; j < K; j++)
            if (dist[(size_t)v * K + j] == INT_MAX) unreached |= 1ull << j;
        if (!unreached) continue;
        u64 hit = 0;
        const int end = g.row_ptr[v + 1];
        for (int e = g.row_ptr[v]; e < end; e++) {
            const int u = g.col[e];
            for (int j = 0; j < K; j++)
                if (((unreached >> j) & 1ull) && dist[(size_t)u * K + j] != INT_MAX) hit |= 1ull << j;
        }
        if (hit) atomic_or_u64(bad, hit);
    }
}

size_t mssssp_work_bytes(const Graph &G, int k) {
    const size_t n = (size_t)G.n;
    return n * (size_t)k * 4 + n * 8 * 3 + n * 4 * 4;
}

// vertex-major distances -> k x n row-major; unreached becomes `unreached`
__global__ __launch_bounds__(kBlock) void k_ms_dist_out(const int32_t *in, int n, int K, int32_t *out,
                                                        int32_t unreached) {
    __shared__ int32_t tile[64][65];
    for (int v0 = blockIdx.x * 64; v0 < n; v0 += gridDim.x * 64) {
        for (int i = threadIdx.x; i < 64 * K; i += kBlock) {
            const int dv = i / K, j = i % K;
            if (v0 + dv < n) tile[j][dv] = in[(size_t)(v0 + dv) * K + j];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * K; i += kBlock) {
            const int j = i / 64, dv = i % 64;
            if (v0 + dv < n) {
                const int32_t x = tile[j][dv];
                out[(size_t)j * n + v0 + dv] = x == INT_MAX ? unreached : x;
            }
        }
        __syncthreads();
    }
}

// The shared loop: UNIT = true is the batched PUSH BFS (depth, -1 unreached),
// false the batched SSSP (distance, INT32_MAX unreached).
static void ms_push_loop(Graph &G, const int32_t *srcs, int k, bool unit, int delta, int32_t *out,
                         hipStream_t stream, gg_stats *st, unsigned long long *overflow_mask) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    if (overflow_mask) *overflow_mask = 0;
    if (k == 0) { scope.finish(); return; }
    require((long long)G.max_degree * 64 < (1ll << 31), GG_ERR_UNSUPPORTED_SCHEDULE,
            "batched push traversal needs max degree below 2^25");
    Lease ws(G);
    const DevGraph g = G.view();
    const int n = g.n;
    ws->aux_i32[3].ensure((size_t)n * k);
    ws->aux_u64[0].ensure(n);
    ws->aux_u64[1].ensure(n);
    ws->aux_u64[2].ensure(n);
    ws->q[0].ensure(n);
    ws->q[1].ensure(n);
    ws->aux_i32[0].ensure(n);
    ws->aux_i32[1].ensure(n > 64 ? n : 64);  // also stages the source list
    ws->counters.ensure(64);
    ws->h_i32.ensure(16);
    ws->h_i64.ensure(2);
    int32_t *ctr = ws->counters.p;
    // the source list is staged in the second far queue: the init kernel reads
    // it before the loop first writes that queue (at the first bucket advance)
    int32_t *dsrc = ws->aux_i32[1].p;
    GG_HIP(hipMemcpyAsync(dsrc, srcs, sizeof(int32_t) * k, hipMemcpyHostToDevice, c.s));
    fill_i32(c, ctr, 64, 0);
    fill_i32(c, ctr + 5, 2, INT_MAX);
    u64 *near0 = ws->aux_u64[0].p, *near1 = ws->aux_u64[1].p, *far = ws->aux_u64[2].p;
    int32_t *dist_vm = ws->aux_i32[3].p;
    hipLaunchKernelGGL(k_mssssp_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, n, k, dsrc, dist_vm,
                       near0, near1, far, ws->q[0].p, ctr, ctr + 12);
    GG_CHECK_LAUNCH();
    c.launches++;
    const void *kern = unit ? (const void *)k_mssssp_fused<true> : (const void *)k_mssssp_fused<false>;
    // wide workgroups: one per compute unit on dense graphs, one per two units
    // on sparse ones, whose rounds are smaller and pay relatively more for the
    // barrier
    const bool sparse = G.m < 8ll * (long long)G.n;
    const int blocks = fused_grid(kern, sparse ? 0 : 1, c.num_cus, kMsBlock);
    MsSsspArgs a{g, k, dist_vm, near0, near1, far, ws->q[0].p, ws->q[1].p, ws->aux_i32[0].p, ws->aux_i32[1].p,
                 ctr, unit ? INT_MAX : delta, prepare_barrier(c, *ws, blocks)};
    void *args[] = {&a};
    launch_cooperative(c, kern, blocks, args, kMsBlock);
    check_barrier(c, *ws);
    GG_HIP(hipMemcpyAsync(ws->h_i32.p, ctr, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    const int32_t *h = ws->h_i32.p;
    require(h[12] == 0, GG_ERR_OUT_OF_MEMORY, "batched traversal queue overflow");
    const int maybe_overflow = unit ? 0 : h[10];
    if (st) {
        st->fused = 1;
        st->iterations = h[8];
        st->push_iterations = h[8];
        st->buckets = unit ? 0 : h[9];
    }
    hipLaunchKernelGGL(k_ms_dist_out, dim3(blocks_for(n, 64, 16384)), dim3(kBlock), 0, c.s, dist_vm, n, k, out,
                       unit ? -1 : INT_MAX);
    GG_CHECK_LAUNCH();
    c.launches++;
    u64 bad = 0;
    if (maybe_overflow) {
        u64 *dbad = (u64 *)(ctr + 32);
        fill_u64(c, dbad, 1, 0ull);
        hipLaunchKernelGGL(k_mssssp_overflow_check, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, g, k,
                           dist_vm, dbad);
        GG_CHECK_LAUNCH();
        c.launches++;
        GG_HIP(hipMemcpyAsync(ws->h_i64.p, dbad, sizeof(u64), hipMemcpyDeviceToHost, c.s));
    }
    GG_HIP(hipStreamSynchronize(c.s));
    if (maybe_overflow) bad = (u64)ws->h_i64.p[0];
    scope.finish();
    if (overflow_mask) *overflow_mask = bad;
    else require(bad == 0, GG_ERR_OVERFLOW, "a shortest-path distance exceeds INT32_MAX-1");
}

void mssssp_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &sch, int32_t *dist, hipStream_t stream,
                gg_stats *st, unsigned long long *overflow_mask) {
    require(G.has_weights, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
    require(sch.s1.delta >= 1, GG_ERR_INVALID_ARG, "delta must be >= 1");
    ms_push_loop(G, srcs, k, false, sch.s1.delta, dist, stream, st, overflow_mask);
}

void msbfs_push_run(Graph &G, const int32_t *srcs, int k, int32_t *depth, hipStream_t stream, gg_stats *st) {
    ms_push_loop(G, srcs, k, true, 0, depth, stream, st, nullptr);
}

}  // namespace gg
