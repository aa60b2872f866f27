// Delta-stepping SSSP on the frontier-driven traversal with a two-bucket
// priority queue (the applyUpdatePriority operator with configDelta in the
// Scheduling Language section; "Active Vertexset Processing Ordering" in the
// GPU Optimization Space section).
//
// Bucket k holds distances in [k*delta, (k+1)*delta). The near queue is the
// frontier of the current bucket; relaxing an edge lowers dist[v] with an
// atomic min, and an improved v goes to the near queue when its new distance
// is still inside the bucket, otherwise to the far queue (deduplicated per
// far epoch). When the near queue drains, the next bucket is the smallest
// floor(dist/delta) over the far entries that lie beyond the current bucket
// (entries that fell back into settled buckets are stale and dropped); the
// far queue is then split into the new near queue and a new far queue.
#include <climits>

#include "algos.hpp"
#include "driver.hpp"
#include "fused.hpp"

namespace gg {

// LDS stage of the far-queue appends (one per kernel)
__device__ __forceinline__ Staged sssp_far_stage(int32_t *farq, int32_t *farc) {
    __shared__ int32_t s_q[kStage];
    __shared__ int s_c;
    return Staged{s_q, &s_c, farq, farc};
}

// STAGE: far appends are staged per workgroup (the load balancer calls
// begin() and flush() at workgroup-uniform points: VP, CM, ETWC and STRICT do)
template <bool STAGE>
struct SsspRelaxT {
    int32_t *dist;
    const uint32_t *w;
    long long bucket_end;   // (k+1)*delta
    int32_t *farq;
    int32_t *farc;
    int32_t far_cap;
    int32_t *far_tag;
    int32_t far_id;
    int32_t *flags;         // [0] distance overflow, [1] far queue overflow
    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    struct Pre { long long nd; int dv; };
    __device__ __forceinline__ Pre load(int u, int v, int e) const {
        return Pre{(long long)dist[u] + (long long)w[e], dist[v]};
    }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, load(u, v, e)); }
    // two-phase form: the atomic minimum's old distance, else the loaded one
    // (no smaller than the candidate then, and a value the compiler cannot
    // fold, so the result test stays out of the atomic's branch)
    using Tok = int;
    __device__ __forceinline__ Tok issue(int, int v, int, const Pre &p, bool ok) const {
        int old = p.dv;
        // a stale (larger) read only costs an atomic
        if (ok && p.nd <= (long long)INT_MAX - 1 && p.nd < p.dv) old = atomic_min_i32(&dist[v], (int)p.nd);
        return old;
    }
    __device__ __forceinline__ int apply(int u, int v, int e, const Pre &p) const {
        return finish(u, v, e, p, true, issue(u, v, e, p, true));
    }
    __device__ __forceinline__ int finish(int, int v, int, const Pre &p, bool ok, Tok old) const {
        const long long nd = p.nd;
        bool to_near = false, to_far = false;
        if (!ok) {
        } else if (nd > (long long)INT_MAX - 1) {
            // not representable: v is unreached so far and may end up with a
            // distance beyond INT32_MAX-1 (confirmed after the loop)
            if (p.dv == INT_MAX) flags[0] = 1;
        } else if (nd < old) {
            if (nd < bucket_end) to_near = true;
            else to_far = far_tag[v] < far_id && atomic_max_i32(&far_tag[v], far_id) < far_id;
        }
        if constexpr (STAGE) stage_append(sssp_far_stage(farq, farc), far_cap, flags + 1, to_far, v);
        else wave_append(farq, farc, far_cap, flags + 1, to_far, v);
        return to_near ? v : -1;
    }
    __device__ __forceinline__ void begin() const {
        if constexpr (STAGE) {
            if (threadIdx.x == 0) *sssp_far_stage(farq, farc).sc = 0;
        }
    }
    __device__ __forceinline__ void flush() const {
        if constexpr (STAGE) {
            __shared__ int s_base;
            stage_flush(sssp_far_stage(farq, farc), far_cap, flags + 1, &s_base);
        }
    }
};
using SsspRelax = SsspRelaxT<false>;

// After the loop: an unreached vertex with a reached neighbour has a true
// distance beyond INT32_MAX-1 (every relaxation into it was unrepresentable).
__global__ __launch_bounds__(kBlock) void k_sssp_overflow_check(DevGraph g, const int32_t *dist, int32_t *flag) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < g.n; v += gridDim.x * kBlock) {
        if (dist[v] != INT_MAX) continue;
        const int end = g.row_ptr[v + 1];
        for (int e = g.row_ptr[v]; e < end; e++)
            if (dist[g.col[e]] != INT_MAX) { *flag = 1; break; }
    }
}

static void confirm_overflow(Ctx &c, const DevGraph &g, const int32_t *dist, int32_t *flag_dev, int32_t *pinned) {
    fill_i32(c, flag_dev, 1, 0);
    hipLaunchKernelGGL(k_sssp_overflow_check, dim3(blocks_for(g.n, kBlock, 8192)), dim3(kBlock), 0, c.s, g, dist,
                       flag_dev);
    GG_CHECK_LAUNCH();
    c.launches++;
    require(read_i32(c, flag_dev, pinned) == 0, GG_ERR_OVERFLOW, "a shortest-path distance exceeds INT32_MAX-1");
}

__global__ __launch_bounds__(kBlock) void k_sssp_init(int32_t *dist, int n, int src, int32_t *q) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) dist[v] = v == src ? 0 : INT_MAX;
    if (blockIdx.x == 0 && threadIdx.x == 0) q[0] = src;
}

// smallest bucket index beyond k among the far entries
__device__ __forceinline__ void far_min_dev(const int32_t *farq, int fc, const int32_t *dist, int delta, int k,
                                            int32_t *kmin, Tid t) {
    int local = INT_MAX;
    const int stride = t.nblocks * kBlock;
    for (int i = t.block * kBlock + (int)threadIdx.x; i < fc; i += stride) {
        const int b = dist[farq[i]] / delta;
        if (b > k && b < local) local = b;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int o = __shfl_xor(local, off, kWave);
        local = o < local ? o : local;
    }
    // a plain read first: once a small bucket index is in, most wavefronts
    // skip the atomic (atomics on one address serialise)
    if (lane_id() == 0 && local != INT_MAX && local < load_relaxed(kmin)) atomic_min_i32(kmin, local);
}

// far entries of bucket knew -> near queue; later buckets -> the next far queue
__device__ __forceinline__ void far_split_dev(const int32_t *farq, int fc, const int32_t *dist, int delta, int knew,
                                              const OutFrontier &near, int32_t *nfarq, int32_t *nfarc, int far_cap,
                                              int32_t *far_tag, int far_id, int32_t *flags, Tid t) {
    // appends staged per workgroup (one global atomic per queue and flush)
    __shared__ StageLDS s_near, s_far;
    if (threadIdx.x == 0) { s_near.c = 0; s_far.c = 0; }
    __syncthreads();
    OutFrontier fo{};
    fo.q = nfarq;
    fo.count = nfarc;
    fo.cap = far_cap;
    fo.overflow = flags + 1;
    const int stride = t.nblocks * kBlock;
    const int n_iter = (fc + stride - 1) / stride;
    for (int it = 0; it < n_iter; it++) {
        const int i = it * stride + t.block * kBlock + (int)threadIdx.x;
        bool to_near = false, to_far = false;
        int v = 0;
        if (i < fc) {
            v = farq[i];
            const int b = dist[v] / delta;
            if (b == knew) to_near = dedup_first<kDedupMonotonic>(near, v);
            else if (b > knew) to_far = atomic_max_i32(&far_tag[v], far_id) < far_id;
        }
        emit_staged<kCreateFused, kDedupNone>(near, s_near, to_near, v);
        emit_staged<kCreateFused, kDedupNone>(fo, s_far, to_far, v);
        if (it % 8 == 7 || it == n_iter - 1) {
            emit_flush<kCreateFused>(near, s_near);
            emit_flush<kCreateFused>(fo, s_far);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_far_min(const int32_t *farq, const int32_t *fc, const int32_t *dist,
                                                    int delta, int k, int32_t *kmin) {
    far_min_dev(farq, *fc, dist, delta, k, kmin, Tid::here());
}

__global__ __launch_bounds__(kBlock) void k_far_split(const int32_t *farq, const int32_t *fc, const int32_t *dist,
                                                      int delta, int knew, OutFrontier near, int32_t *nfarq,
                                                      int32_t *nfarc, int far_cap, int32_t *far_tag, int far_id,
                                                      int32_t *flags) {
    far_split_dev(farq, *fc, dist, delta, knew, near, nfarq, nfarc, far_cap, far_tag, far_id, flags, Tid::here());
}

// ---- fused: the bucket loop in one persistent launch ---------------------------------
// ctr[0..2] rotating near sizes, ctr[3..4] far sizes, ctr[5..6] bucket minima,
// ctr[8] relax rounds, ctr[9] buckets, ctr[10..11] flags, ctr[12] near overflow
struct FusedSsspArgs {
    DevGraph g;
    int32_t *dist;
    int32_t *q0, *q1;
    int32_t *farq0, *farq1;
    int32_t *ctr;
    int32_t *near_tag, *far_tag;
    int32_t qcap;
    int32_t delta;
    GridBarrier bar;
    unsigned long long *ecount;
    long long *scan, *scan_part;  // STRICT: the near queue's degree scan and per-workgroup sums
};

template <int LB>
__global__ __launch_bounds__(kBlock) void k_sssp_fused(FusedSsspArgs a) {
    const Tid t = Tid::here();
    long long ne = 0;
    GridBarrier bar = a.bar;
    int32_t *qin = a.q0, *qout = a.q1;
    int r = 0, k = 0, fe = 0, adv = 0, rounds = 0;
    int32_t *flags = a.ctr + 10;
    const bool lead = t.block == 0 && threadIdx.x == 0;
    for (;;) {
        const int cnt = load_relaxed(&a.ctr[r % 3]);
        if (lead) __hip_atomic_store(&a.ctr[(r + 2) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        OutFrontier o{};
        o.q = qout;
        o.count = &a.ctr[(r + 1) % 3];
        o.cap = a.qcap;
        o.overflow = a.ctr + 12;
        o.tags = a.near_tag;
        o.iter = r + 1;
        int32_t *farq = (fe & 1) ? a.farq1 : a.farq0;
        int32_t *farc = a.ctr + 3 + (fe & 1);
        if (cnt > 0) {
            SsspRelax f{a.dist, a.g.w, (long long)(k + 1) * a.delta, farq, farc, a.g.n, a.far_tag, fe + 1, flags};
            const SrcQueue src{qin, cnt};
            if constexpr (LB == GG_LB_VERTEX_BASED) lb_vp<kCreateFused, kDedupMonotonic, false>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_WM) lb_wm<kCreateFused, kDedupMonotonic>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_CM) lb_cm<kCreateFused, kDedupMonotonic, false>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_STRICT) {
                if (!grid_degree_scan(a.g, src, a.scan, a.scan_part, bar)) break;
                lb_strict<kCreateFused, kDedupMonotonic>(a.g, src, a.scan, f, o, t, ne);
            } else lb_etwc<kCreateFused, kDedupMonotonic, false>(a.g, src, f, o, t, ne);
            rounds++;
        } else {
            const int fc = load_relaxed(farc);
            if (fc == 0) break;
            int32_t *kmin = a.ctr + 5 + (adv & 1);
            if (lead) {
                __hip_atomic_store(a.ctr + 5 + ((adv + 1) & 1), INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(a.ctr + 3 + ((fe + 1) & 1), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            far_min_dev(farq, fc, a.dist, a.delta, k, kmin, t);
            if (!grid_sync(bar)) break;
            const int knew = load_relaxed(kmin);
            if (knew == INT_MAX) break;
            int32_t *nfarq = (fe & 1) ? a.farq0 : a.farq1;
            far_split_dev(farq, fc, a.dist, a.delta, knew, o, nfarq, a.ctr + 3 + ((fe + 1) & 1), a.g.n, a.far_tag,
                          fe + 2, flags, t);
            fe++;
            adv++;
            k = knew;
        }
        if (!grid_sync(bar)) break;
        int32_t *tq = qin; qin = qout; qout = tq;
        r++;
    }
    if (lead) { a.ctr[8] = rounds; a.ctr[9] = adv + 1; }
    flush_edge_count(ne, a.ecount);
}

static void sssp_fused(Ctx &c, Graph &G, Workspace &ws, int32_t src, const gg_simple_schedule &s, int32_t *dist,
                       gg_stats *st) {
    const DevGraph g = G.view();
    const void *kern = nullptr;
    switch (s.load_balance) {
    case GG_LB_VERTEX_BASED: kern = (const void *)k_sssp_fused<GG_LB_VERTEX_BASED>; break;
    case GG_LB_WM: kern = (const void *)k_sssp_fused<GG_LB_WM>; break;
    case GG_LB_CM: kern = (const void *)k_sssp_fused<GG_LB_CM>; break;
    case GG_LB_ETWC: kern = (const void *)k_sssp_fused<GG_LB_ETWC>; break;
    case GG_LB_STRICT: kern = (const void *)k_sssp_fused<GG_LB_STRICT>; break;
    default: throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, "kernel fusion supports VERTEX_BASED, WM, CM, ETWC and STRICT");
    }
    const int n = g.n;
    ws.q[0].ensure(n);
    ws.q[1].ensure(n);
    ws.aux_i32[0].ensure(n);
    ws.aux_i32[1].ensure(n);
    ws.aux_i32[2].ensure(n);
    ws.tags.ensure(n);
    ws.counters.ensure(64);
    ws.h_i32.ensure(16);
    fill_i32(c, ws.counters.p, 64, 0);
    fill_i32(c, ws.counters.p + 5, 2, INT_MAX);
    fill_i32(c, ws.tags.p, n, 0);
    fill_i32(c, ws.aux_i32[2].p, n, 0);
    hipLaunchKernelGGL(k_sssp_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, dist, n, src, ws.q[0].p);
    GG_CHECK_LAUNCH();
    c.launches++;
    fill_i32(c, ws.counters.p, 1, 1);
    const int blocks = fused_grid_for(kern, G, c.num_cus);
    if (s.load_balance == GG_LB_STRICT) {
        ws.scan.ensure((size_t)n + 1);
        ws.scan_part.ensure((size_t)blocks);
    }
    FusedSsspArgs a{g, dist, ws.q[0].p, ws.q[1].p, ws.aux_i32[0].p, ws.aux_i32[1].p, ws.counters.p, ws.tags.p,
                    ws.aux_i32[2].p, n, s.delta, prepare_barrier(c, ws, blocks), c.edge_counter, ws.scan.p,
                    ws.scan_part.p};
    void *args[] = {&a};
    launch_cooperative(c, kern, blocks, args);
    check_barrier(c, ws);
    GG_HIP(hipMemcpyAsync(ws.h_i32.p, ws.counters.p, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    const int32_t *h = ws.h_i32.p;
    require(h[11] == 0 && h[12] == 0, GG_ERR_OUT_OF_MEMORY, "SSSP queue overflow");
    const int maybe_overflow = h[10];
    if (st) {
        st->fused = 1;
        st->iterations = h[8];
        st->push_iterations = h[8];
        st->buckets = h[9];
    }
    if (maybe_overflow) confirm_overflow(c, g, dist, ws.counters.p + 13, ws.h_i32.p);
}

// Dense rounds over the EdgeBlocked COO (a hybrid schedule's s2 of EDGE_ONLY
// with EdgeBlocking): every edge of one destination segment whose source is
// in the input frontier (a bitmap) is relaxed, kEdgeBatch edges per lane in
// flight. f reads the weights in the blocked order (its w is the layout's).
// A launch's distance reads and minima stay inside one segment's entries.
template <int CREATE, int DEDUP>
__global__ __launch_bounds__(kBlock) void k_sssp_push_blocked(const int32_t *src, const int32_t *dst, long long lo,
                                                              long long hi, const unsigned long long *member,
                                                              SsspRelaxT<false> f, OutFrontier out,
                                                              unsigned long long *ecount) {
    // queue appends staged per workgroup (one global atomic per flush): a
    // dense round appends a large share of the graph's vertices
    __shared__ StageLDS s_st;
    if (threadIdx.x == 0) s_st.c = 0;
    __syncthreads();
    const long long stride = (long long)gridDim.x * kBlock;
    long long ne = 0;
    for (long long base = lo + (long long)blockIdx.x * kBlock; base < hi; base += kEdgeBatch * stride) {
        const long long e0 = base + threadIdx.x;
        int uu[kEdgeBatch], vv[kEdgeBatch];
        bool take[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) {
            const long long e = e0 + b * stride;
            uu[b] = src[e < hi ? e : hi - 1];
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) take[b] = e0 + b * stride < hi && bit_test(member, uu[b]);
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) vv[b] = take[b] ? dst[e0 + b * stride] : 0;
        SsspRelaxT<false>::Pre pre[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++)
            pre[b] = take[b] ? f.load(uu[b], vv[b], (int)(e0 + b * stride)) : SsspRelaxT<false>::Pre{0, 0};
        int ee[kEdgeBatch], xx[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) ee[b] = (int)(e0 + b * stride);
        apply_batch<kEdgeBatch>(f, uu, vv, ee, pre, take, xx, ne);
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) emit_staged<CREATE, DEDUP>(out, s_st, xx[b] >= 0, xx[b]);
        emit_flush_half<CREATE>(out, s_st);
    }
    emit_flush<CREATE>(out, s_st);
    flush_edge_count(ne, ecount);
}

template <int CREATE, int DEDUP>
static void launch_blocked(Ctx &c, const EdgeBlocked &eb, const unsigned long long *member,
                           const SsspRelaxT<false> &f, const OutFrontier &o) {
    for (size_t sg = 0; sg + 1 < eb.seg_start.size(); sg++) {
        const long long lo = eb.seg_start[sg], hi = eb.seg_start[sg + 1];
        if (hi <= lo) continue;
        hipLaunchKernelGGL((k_sssp_push_blocked<CREATE, DEDUP>),
                           dim3(blocks_for((hi - lo + kEdgeBatch - 1) / kEdgeBatch, kBlock, 16384)), dim3(kBlock), 0,
                           c.s, eb.src.p, eb.dst.p, lo, hi, member, f, o, c.edge_counter);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
}

static void sssp_blocked_step(Ctx &c, const EdgeBlocked &eb, const unsigned long long *member, int create, int dd,
                              const SsspRelaxT<false> &f, const OutFrontier &o) {
    if (create == kCreateBoolmap) launch_blocked<kCreateBoolmap, kDedupNone>(c, eb, member, f, o);
    else if (create == kCreateBitmap) launch_blocked<kCreateBitmap, kDedupNone>(c, eb, member, f, o);
    else if (dd == kDedupMonotonic) launch_blocked<kCreateFused, kDedupMonotonic>(c, eb, member, f, o);
    else if (dd == kDedupBitmap) launch_blocked<kCreateFused, kDedupBitmap>(c, eb, member, f, o);
    else if (dd == kDedupBoolmap) launch_blocked<kCreateFused, kDedupBoolmap>(c, eb, member, f, o);
    else launch_blocked<kCreateFused, kDedupNone>(c, eb, member, f, o);
}

static const EdgeBlocked &blocked_layout(Ctx &c, Graph &G, int32_t N) {
    edgeblock_prepare(c, G, N);
    std::lock_guard<std::mutex> lk(G.mu);
    const EdgeBlocked &eb = *G.eb.at(N);
    require(eb.w.p != nullptr || G.m == 0, GG_ERR_INVALID_ARG, "EdgeBlocked layout has no weights");
    return eb;
}

void sssp_run(Graph &G, int32_t src, const gg_schedule &sch, int32_t *dist, hipStream_t stream, gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    Lease ws(G);
    // s1 fixes the loop (delta, fusion); a hybrid schedule runs s2 in rounds
    // whose input frontier holds more than threshold * n vertices
    const gg_simple_schedule &s = sch.s1;
    const bool hyb = sch.hybrid != 0;
    if ((s.load_balance == GG_LB_EDGE_ONLY && !s.edge_blocking) ||
        (hyb && sch.s2.load_balance == GG_LB_EDGE_ONLY && !sch.s2.edge_blocking))
        ensure_coo(c, G);
    const DevGraph g = G.view();
    const int n = g.n;
    if (s.kernel_fusion) {
        sssp_fused(c, G, *ws, src, s, dist, st);
        scope.finish();
        return;
    }
    const int dd = dedup_mode(s);
    const bool nodedup = dd == kDedupNone || (hyb && sch.s2.frontier_creation == GG_CREATE_FUSED &&
                                             dedup_mode(sch.s2) == kDedupNone);
    const long long qcap = nodedup ? (long long)n + g.m : (long long)n;
    const EdgeBlocked *eb = nullptr;
    FrontierState fs(c, *ws, n, qcap);
    ws->tags.ensure(n);
    fill_i32(c, ws->tags.p, n, 0);
    ws->aux_i32[0].ensure(n);  // far queues
    ws->aux_i32[1].ensure(n);
    ws->aux_i32[2].ensure(n);  // far tags
    fill_i32(c, ws->aux_i32[2].p, n, 0);
    int32_t *farq[2] = {ws->aux_i32[0].p, ws->aux_i32[1].p};
    int32_t *ctr = ws->counters.p;  // [16..17] far sizes, [18] bucket min, [20..21] flags
    hipLaunchKernelGGL(k_sssp_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, dist, n, src,
                       fs.queue());
    GG_CHECK_LAUNCH();
    c.launches++;
    fs.count = 1;
    int k = 0, fe = 0, iter = 1, buckets = 1, maybe_overflow = 0;
    const int delta = s.delta;
    for (;;) {
        while (fs.count > 0) {
            if (st) { st->vertices_processed += fs.count; st->iterations++; st->push_iterations++; }
            const gg_simple_schedule &sr = hyb && (double)fs.count > (double)sch.threshold * n ? sch.s2 : s;
            const int ddr = dedup_mode(sr);
            if (sr.load_balance == GG_LB_EDGE_ONLY && sr.edge_blocking) {
                if (eb == nullptr) eb = &blocked_layout(c, G, sr.blocking_size);
                const unsigned long long *member = fs.as_bitmap();
                OutFrontier o = fs.prep_out(sr.frontier_creation, ddr, iter++);
                SsspRelaxT<false> f{dist, eb->w.p, (long long)(k + 1) * delta, farq[fe & 1], ctr + 16 + (fe & 1), n,
                                    ws->aux_i32[2].p, fe + 1, ctr + 20};
                sssp_blocked_step(c, *eb, member, sr.frontier_creation, ddr, f, o);
                fs.commit(sr.frontier_creation);
                continue;
            }
            const int32_t *q = fs.as_queue();
            OutFrontier o = fs.prep_out(sr.frontier_creation, ddr, iter++, sr.load_balance);
            const PushPlan plan{sr.load_balance, sr.frontier_creation, ddr};
            const int lbm = sr.load_balance;
            if (lbm == GG_LB_STRICT || lbm == GG_LB_CM || lbm == GG_LB_ETWC || lbm == GG_LB_VERTEX_BASED) {
                SsspRelaxT<true> f{dist, g.w, (long long)(k + 1) * delta, farq[fe & 1], ctr + 16 + (fe & 1), n,
                                   ws->aux_i32[2].p, fe + 1, ctr + 20};
                push_apply(c, g, *ws, plan, q, fs.count, f, o, member_map(*ws, n, sr.load_balance));
            } else {
                SsspRelax f{dist, g.w, (long long)(k + 1) * delta, farq[fe & 1], ctr + 16 + (fe & 1), n,
                            ws->aux_i32[2].p, fe + 1, ctr + 20};
                push_apply(c, g, *ws, plan, q, fs.count, f, o, member_map(*ws, n, sr.load_balance));
            }
            fs.commit(sr.frontier_creation);
        }
        GG_HIP(hipMemcpyAsync(ws->h_i32.p, ctr + 16, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
        GG_HIP(hipStreamSynchronize(c.s));
        require(ws->h_i32.p[5] == 0, GG_ERR_OUT_OF_MEMORY, "far queue overflow");
        maybe_overflow |= ws->h_i32.p[4];
        const int fc = ws->h_i32.p[fe & 1];
        if (fc == 0) break;
        fill_i32(c, ctr + 18, 1, INT_MAX);
        hipLaunchKernelGGL(k_far_min, dim3(blocks_for(fc, kBlock * 4, 1024)), dim3(kBlock), 0, c.s, farq[fe & 1],
                           ctr + 16 + (fe & 1), dist, delta, k, ctr + 18);
        GG_CHECK_LAUNCH();
        c.launches++;
        const int knew = read_i32(c, ctr + 18, ws->h_i32.p + 8);
        if (knew == INT_MAX) break;
        fill_i32(c, ctr + 16 + ((fe + 1) & 1), 1, 0);
        OutFrontier o = fs.prep_out(kCreateFused, kDedupMonotonic, iter++);
        o.tags = ws->tags.p;
        hipLaunchKernelGGL(k_far_split, dim3(blocks_for(fc, kBlock * 8, 1024)), dim3(kBlock), 0, c.s, farq[fe & 1],
                           ctr + 16 + (fe & 1), dist, delta, knew, o, farq[(fe + 1) & 1], ctr + 16 + ((fe + 1) & 1), n,
                           ws->aux_i32[2].p, fe + 2, ctr + 20);
        GG_CHECK_LAUNCH();
        c.launches++;
        fs.commit(kCreateFused);
        fe++;
        k = knew;
        buckets++;
    }
    if (st) st->buckets = buckets;
    if (maybe_overflow) confirm_overflow(c, g, dist, ctr + 22, ws->h_i32.p + 9);
    scope.finish();
}

}  // namespace gg
