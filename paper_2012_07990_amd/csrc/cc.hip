// Connected components by hooking and shortcutting (the Soman et al.
// algorithm the paper's Evaluation section names for CC). Each round sweeps
// every edge (u, v) with the schedule's load balancer: when the labels of
// the endpoints differ, the larger label's entry is lowered to the smaller
// one with an atomic min (hooking); then every label is replaced by the root
// it reaches (shortcutting). Rounds repeat until a sweep hooks nothing. Labels
// only decrease and never leave the component, so the fixpoint labels every
// vertex with the smallest id of its component.
#include <algorithm>
#include <vector>

#include "algos.hpp"
#include "driver.hpp"
#include "fused.hpp"

namespace gg {

struct CcHook {
    int32_t *label;
    int32_t *changed;
    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    // the last hook this lane made: label[m_hi] <= m_lo holds from then on
    // (labels only decrease), so a hook of m_hi to a value >= m_lo is a no-op
    // and is skipped -- the lanes sharing a hub's edges would otherwise all
    // hit the hub's label with atomics
    mutable int m_hi = -1, m_lo = 0;
    struct Pre { int lu, lv; };
    __device__ __forceinline__ Pre load(int u, int v, int) const { return Pre{label[u], v < u ? 0 : label[v]}; }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, load(u, v, e)); }
    __device__ __forceinline__ int apply(int u, int v, int, const Pre &p) const {
        if (v < u) return -1;  // symmetric graph: every undirected edge once
        const int lu = p.lu, lv = p.lv;  // stale labels only delay a hook to a later round
        bool ch = false;
        if (lu != lv) {
            const int hi = lu > lv ? lu : lv, lo = lu > lv ? lv : lu;
            if (hi != m_hi || lo < m_lo) {
                // a plain read first: labels hit by many hooks (component roots)
                // drop early, and later hooks see that and skip the atomic
                // (a stale, larger read only costs the atomic)
                if (label[hi] > lo) ch = atomic_min_i32(&label[hi], lo) > lo;
                m_hi = hi;
                m_lo = lo;
            }
        }
        // one store per wavefront to the shared flag, and none once it is seen set
        const uint64_t m = __ballot(ch);
        if (m && lane_id() == first_lane(m) && load_relaxed(changed) == 0) *changed = 1;
        return -1;
    }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};

// EDGE_ONLY on a symmetric graph: every undirected edge once, as the pairs
// (u, v) with u < v (the hook ignores the mirrored entries anyway), each lane
// loading kEdgeBatch pairs and their labels before hooking any of them
__global__ __launch_bounds__(kBlock) void k_cc_hook_pairs(const int2 *pairs, long long np, CcHook f,
                                                          unsigned long long *ecount) {
    const long long stride = (long long)gridDim.x * kBlock;
    long long ne = 0;
    for (long long e0 = (long long)blockIdx.x * kBlock + threadIdx.x; e0 < np; e0 += kEdgeBatch * stride) {
        int2 pp[kEdgeBatch];
        CcHook::Pre pre[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) {
            const long long e = e0 + b * stride;
            // one 8-byte non-temporal load per pair (x in the low word)
            const unsigned long long w = __builtin_nontemporal_load(
                reinterpret_cast<const unsigned long long *>(pairs) + (e < np ? e : np - 1));
            pp[b] = make_int2((int)(unsigned)w, (int)(unsigned)(w >> 32));
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) pre[b] = f.load(pp[b].x, pp[b].y, 0);
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) {
            const bool live = e0 + b * stride < np;
            // a lane past the end repeats the last pair: the hook is idempotent
            f.apply(pp[b].x, pp[b].y, 0, pre[b]);
            ne += live;
        }
    }
    flush_edge_count(ne, ecount);
}

// per vertex: the number of its neighbours above it (rows are sorted)
__global__ __launch_bounds__(kBlock) void k_upper_count(const int32_t *rp, const int32_t *col, int n, int32_t *cnt) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        int lo = rp[v], hi = rp[v + 1];
        const int end = hi;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (col[mid] <= v) lo = mid + 1; else hi = mid;
        }
        cnt[v] = end - lo;
    }
}

// one wavefront per vertex copies its upper neighbours as pairs
__global__ __launch_bounds__(kBlock) void k_upper_fill(const int32_t *rp, const int32_t *col, int n,
                                                      const int32_t *off, int2 *pairs) {
    const int wpb = kBlock / kWave;
    for (int v = blockIdx.x * wpb + threadIdx.x / kWave; v < n; v += gridDim.x * wpb) {
        const int end = rp[v + 1], cntv = off[v + 1] - off[v];
        const int first = end - cntv;
        for (int i = lane_id(); i < cntv; i += kWave) pairs[off[v] + i] = make_int2(v, col[first + i]);
    }
}

// Built once per graph under its lock and completed before the lock is
// released (a query on another stream that finds it present reads a
// finished list).
static void ensure_upper(Ctx &c, Graph &G) {
    std::lock_guard<std::mutex> lk(G.mu);
    if (G.upper.p) return;
    const int n = G.n;
    DevBuf<int32_t> off;
    DevBuf<long long> part;
    off.ensure((size_t)n + 1);
    part.ensure(exclusive_scan_partials(n));
    hipLaunchKernelGGL(k_upper_count, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, G.row_ptr.p,
                       G.col.p, n, off.p);
    GG_CHECK_LAUNCH();
    exclusive_scan_i32(c, off.p, n, part.p);
    int32_t total = 0;
    GG_HIP(hipMemcpyAsync(&total, off.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    DevBuf<int2> pairs;
    pairs.ensure((size_t)std::max(total, 1));
    hipLaunchKernelGGL(k_upper_fill, dim3(blocks_for(n, kBlock / kWave, 16384)), dim3(kBlock), 0, c.s,
                       G.row_ptr.p, G.col.p, n, off.p, pairs.p);
    GG_CHECK_LAUNCH();
    GG_HIP(hipStreamSynchronize(c.s));
    c.launches += 3;
    G.m_upper = total;
    std::swap(G.upper.p, pairs.p);
    std::swap(G.upper.n, pairs.n);
}

// ---- EdgeBlocking of the pair list ---------------------------------------------
// The hook sweep processes every undirected edge each round, which is where
// the EdgeBlocking preprocessing applies: the pairs are grouped by the
// segment floor(v / N) of their larger endpoint, keeping CSR order inside a
// segment, and each segment is swept by its own launch, so the random label
// reads of a launch stay inside one segment's labels (and its L2 lines) while
// the smaller endpoints stream through label[] in ascending order. A stable
// counting sort on the device: per tile of kPairTile pairs a histogram over
// the S <= kMaxPairSeg segments, an exclusive scan of the histograms in
// segment-major order, then each tile scatters its pairs in order, ranking
// equal segments within a wavefront by matching the six bits of the
// segment id with ballots.
constexpr int kPairTile = kBlock * 8;
constexpr int kMaxPairSeg = 64;

__global__ __launch_bounds__(kBlock) void k_pair_seg_hist(const int2 *pairs, long long np, int N, int S, long long T,
                                                          int32_t *hist) {
    __shared__ int h[kMaxPairSeg];
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        for (int i = threadIdx.x; i < S; i += kBlock) h[i] = 0;
        __syncthreads();
        const long long lo = t * kPairTile, hi = lo + kPairTile < np ? lo + kPairTile : np;
        for (long long i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&h[pairs[i].y / N], 1);
        __syncthreads();
        for (int i = threadIdx.x; i < S; i += kBlock) hist[(long long)i * T + t] = h[i];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_pair_seg_scatter(const int2 *pairs, long long np, int N, int S,
                                                             long long T, const int32_t *off, int2 *out) {
    __shared__ int run[kMaxPairSeg];
    __shared__ int wcnt[kBlock / kWave][kMaxPairSeg];
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        for (int i = tid; i < S; i += kBlock) run[i] = off[(long long)i * T + t];
        const long long lo = t * kPairTile, hi = lo + kPairTile < np ? lo + kPairTile : np;
        for (long long base = lo; base < hi; base += kBlock) {
            const long long i = base + tid;
            const bool live = i < hi;
            const int2 p = live ? pairs[i] : make_int2(0, 0);
            const int s = live ? p.y / N : 0;
            uint64_t same = __ballot(live);
#pragma unroll
            for (int b = 0; b < 6; b++) {
                const bool bit = (s >> b) & 1;
                const uint64_t m = __ballot(live && bit);
                same &= bit ? m : ~m;
            }
            const int below = lanes_below(same);
            for (int k = tid; k < (kBlock / kWave) * S; k += kBlock) wcnt[k / S][k % S] = 0;
            __syncthreads();
            if (live && below == 0) wcnt[w][s] = __popcll(same);
            __syncthreads();
            if (live) {
                int pos = run[s] + below;
                for (int w2 = 0; w2 < w; w2++) pos += wcnt[w2][s];
                out[pos] = p;
            }
            __syncthreads();
            for (int k = tid; k < S; k += kBlock) {
                int tot = 0;
                for (int w2 = 0; w2 < kBlock / kWave; w2++) tot += wcnt[w2][k];
                run[k] += tot;
            }
            __syncthreads();
        }
    }
}

// the pair list blocked by segments of N vertices, built once per (graph, N)
static const BlockedPairs &ensure_upper_blocked(Ctx &c, Graph &G, int32_t N) {
    {
        std::lock_guard<std::mutex> lk(G.mu);
        auto it = G.upper_eb.find(N);
        if (it != G.upper_eb.end()) return *it->second;
    }
    const long long np = G.m_upper;
    const int S = (int)(((long long)G.n + N - 1) / N);
    require(S >= 1 && S <= kMaxPairSeg, GG_ERR_UNSUPPORTED_SCHEDULE,
            "CC EdgeBlocking supports at most 64 segments (blocking_size >= n / 64)");
    auto b = std::make_unique<BlockedPairs>();
    b->N = N;
    b->pairs.ensure((size_t)std::max<long long>(np, 1));
    b->seg_start.assign((size_t)S + 1, np);
    if (np > 0) {
        const long long T = (np + kPairTile - 1) / kPairTile;
        require((long long)S * T < (1ll << 31) - 1, GG_ERR_INVALID_ARG, "pair list too large");
        const int hn = (int)(S * T);
        DevBuf<int32_t> off;
        DevBuf<long long> part;
        off.ensure((size_t)hn + 1);
        part.ensure(exclusive_scan_partials(hn));
        const unsigned grid = (unsigned)std::min<long long>(T, 8192);
        hipLaunchKernelGGL(k_pair_seg_hist, dim3(grid), dim3(kBlock), 0, c.s, G.upper.p, np, N, S, T, off.p);
        GG_CHECK_LAUNCH();
        exclusive_scan_i32(c, off.p, hn, part.p);
        hipLaunchKernelGGL(k_pair_seg_scatter, dim3(grid), dim3(kBlock), 0, c.s, G.upper.p, np, N, S, T, off.p,
                           b->pairs.p);
        GG_CHECK_LAUNCH();
        c.launches += 3;
        std::vector<int32_t> starts((size_t)S);
        for (int s = 0; s < S; s++)
            GG_HIP(hipMemcpyAsync(&starts[s], off.p + (size_t)s * T, sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
        GG_HIP(hipStreamSynchronize(c.s));
        for (int s = 0; s < S; s++) b->seg_start[s] = starts[s];
    }
    std::lock_guard<std::mutex> lk(G.mu);
    auto &slot = G.upper_eb[N];
    if (!slot) slot = std::move(b);
    return *slot;
}

__global__ __launch_bounds__(kBlock) void k_cc_init(int32_t *label, int32_t *ids, int n) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        label[v] = v;
        ids[v] = v;
    }
}

__device__ __forceinline__ void cc_compress_dev(int32_t *label, int n, Tid t) {
    for (int v = t.block * kBlock + (int)threadIdx.x; v < n; v += t.nblocks * kBlock) {
        int l = label[v];
        for (;;) {
            const int ll = label[l];
            if (ll == l) break;
            l = ll;
        }
        label[v] = l;
    }
}

__global__ __launch_bounds__(kBlock) void k_cc_compress(int32_t *label, int n) {
    cc_compress_dev(label, n, Tid::here());
}

// ---- fused: hook / barrier / shortcut / barrier in one persistent launch ----
struct FusedCcArgs {
    DevGraph g;
    int32_t *label;
    int32_t *ids;
    int32_t *ctr;  // [0..2] changed flags (rotating), [3] rounds
    GridBarrier bar;
    unsigned long long *ecount;
    long long *scan, *scan_part;  // STRICT: the degree scan of every vertex (computed once)
};

template <int LB>
__global__ __launch_bounds__(kBlock) void k_cc_fused(FusedCcArgs a) {
    const Tid t = Tid::here();
    long long ne = 0;
    GridBarrier bar = a.bar;
    const SrcQueue src{a.ids, a.g.n};
    OutFrontier o{};  // hooks emit nothing
    int r = 0;
    bool ok = true;
    if constexpr (LB == GG_LB_STRICT) ok = grid_degree_scan(a.g, src, a.scan, a.scan_part, bar);
    for (; ok;) {
        // round r hooks into flag r%3 and everyone reads it after the second
        // barrier; flag (r+1)%3 was last read before round r-1's barriers
        int32_t *changed = a.ctr + (r % 3);
        if (t.block == 0 && threadIdx.x == 0)
            __hip_atomic_store(a.ctr + ((r + 1) % 3), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        CcHook f{a.label, changed};
        if constexpr (LB == GG_LB_VERTEX_BASED) lb_vp<kCreateBoolmap, kDedupNone, false>(a.g, src, f, o, t, ne);
        else if constexpr (LB == GG_LB_WM) lb_wm<kCreateBoolmap, kDedupNone>(a.g, src, f, o, t, ne);
        else if constexpr (LB == GG_LB_CM) lb_cm<kCreateBoolmap, kDedupNone, false>(a.g, src, f, o, t, ne);
        else if constexpr (LB == GG_LB_STRICT) lb_strict<kCreateBoolmap, kDedupNone>(a.g, src, a.scan, f, o, t, ne);
        else lb_etwc<kCreateBoolmap, kDedupNone, false>(a.g, src, f, o, t, ne);
        if (!grid_sync(bar)) break;
        cc_compress_dev(a.label, a.g.n, t);
        if (!grid_sync(bar)) break;
        r++;
        if (load_relaxed(changed) == 0) break;
    }
    if (t.block == 0 && threadIdx.x == 0) a.ctr[3] = r;
    flush_edge_count(ne, a.ecount);
}

void cc_run(Graph &G, const gg_schedule &sch, int32_t *label, hipStream_t stream, gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    Lease ws(G);
    const gg_simple_schedule &s = sch.s1;
    if (s.load_balance == GG_LB_EDGE_ONLY && !G.symmetric) ensure_coo(c, G);
    const DevGraph g = G.view();
    const int n = g.n;
    ws->aux_i32[0].ensure(n);  // identity frontier: every vertex is a source each round
    ws->counters.ensure(64);
    ws->h_i32.ensure(16);
    fill_i32(c, ws->counters.p, 64, 0);
    hipLaunchKernelGGL(k_cc_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, label,
                       ws->aux_i32[0].p, n);
    GG_CHECK_LAUNCH();
    c.launches++;
    if (s.kernel_fusion) {
        const void *kern = nullptr;
        switch (s.load_balance) {
        case GG_LB_VERTEX_BASED: kern = (const void *)k_cc_fused<GG_LB_VERTEX_BASED>; break;
        case GG_LB_WM: kern = (const void *)k_cc_fused<GG_LB_WM>; break;
        case GG_LB_CM: kern = (const void *)k_cc_fused<GG_LB_CM>; break;
        case GG_LB_ETWC: kern = (const void *)k_cc_fused<GG_LB_ETWC>; break;
        case GG_LB_STRICT: kern = (const void *)k_cc_fused<GG_LB_STRICT>; break;
        default:
            throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, "kernel fusion supports VERTEX_BASED, WM, CM, ETWC and STRICT");
        }
        const int blocks = fused_grid_for(kern, G, c.num_cus);
        if (s.load_balance == GG_LB_STRICT) {
            ws->scan.ensure((size_t)n + 1);
            ws->scan_part.ensure((size_t)blocks);
        }
        FusedCcArgs a{g,          label, ws->aux_i32[0].p, ws->counters.p, prepare_barrier(c, *ws, blocks),
                      c.edge_counter, ws->scan.p, ws->scan_part.p};
        void *args[] = {&a};
        launch_cooperative(c, kern, blocks, args);
        check_barrier(c, *ws);
        if (st) {
            st->fused = 1;
            st->iterations = read_i32(c, ws->counters.p + 3, ws->h_i32.p);
            st->push_iterations = st->iterations;
        }
        scope.finish();
        return;
    }
    if (s.load_balance == GG_LB_EDGE_ONLY && G.symmetric) {
        ensure_upper(c, G);
        const long long np = G.m_upper;
        // one sweep per segment of the blocked list, else one over the whole list
        const int2 *pairs = G.upper.p;
        std::vector<long long> seg{0, np};
        if (s.edge_blocking) {
            const BlockedPairs &bp = ensure_upper_blocked(c, G, s.blocking_size);
            pairs = bp.pairs.p;
            seg = bp.seg_start;
        }
        for (;;) {
            fill_i32(c, ws->counters.p, 1, 0);
            for (size_t k = 0; k + 1 < seg.size(); k++) {
                const long long cnt = seg[k + 1] - seg[k];
                if (cnt <= 0) continue;
                hipLaunchKernelGGL(k_cc_hook_pairs,
                                   dim3(blocks_for((cnt + kEdgeBatch - 1) / kEdgeBatch, kBlock, 16384)), dim3(kBlock),
                                   0, c.s, pairs + seg[k], cnt, CcHook{label, ws->counters.p}, c.edge_counter);
                GG_CHECK_LAUNCH();
                c.launches++;
            }
            hipLaunchKernelGGL(k_cc_compress, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, label, n);
            GG_CHECK_LAUNCH();
            c.launches++;
            if (st) { st->iterations++; st->push_iterations++; st->vertices_processed += n; }
            if (read_i32(c, ws->counters.p, ws->h_i32.p) == 0) break;
        }
        scope.finish();
        return;
    }
    // the hooks emit nothing: a dense output map receives no writes
    ws->boolmap[0].ensure(((size_t)n + 255) / 256 * 256);
    OutFrontier o{};
    o.boolmap = ws->boolmap[0].p;
    const PushPlan p{s.load_balance, kCreateBoolmap, kDedupNone};
    for (;;) {
        fill_i32(c, ws->counters.p, 1, 0);
        push_apply(c, g, *ws, p, ws->aux_i32[0].p, n, CcHook{label, ws->counters.p}, o,
                   member_map(*ws, n, s.load_balance));
        hipLaunchKernelGGL(k_cc_compress, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, label, n);
        GG_CHECK_LAUNCH();
        c.launches++;
        if (st) { st->iterations++; st->push_iterations++; st->vertices_processed += n; }
        if (read_i32(c, ws->counters.p, ws->h_i32.p) == 0) break;
    }
    scope.finish();
}

}  // namespace gg
