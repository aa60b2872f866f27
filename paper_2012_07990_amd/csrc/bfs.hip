// BFS on the frontier-driven edgeset.apply (the BFS program of the paper's
// Algorithm Language section, with the direction-optimising schedule of its
// Scheduling Language section). The update is the compare-and-swap rewrite
// of "parent[dst] = src" that the paper's PUSH schedule generates, storing
// the level instead of the parent (the level is the unique part of the
// result); PULL scans a vertex's neighbours for a member of the input
// frontier and stops at the first one, without atomics.
#include "algos.hpp"
#include "bfs.hpp"
#include "driver.hpp"
#include "fused.hpp"

namespace gg {

__global__ __launch_bounds__(kBlock) void k_bfs_init(int32_t *depth, int n, int src, int32_t *q) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) depth[v] = v == src ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) q[0] = src;
}

// PULL: one lane per destination v; input frontier probed as a boolmap or
// bitmap; the output frontier is written whole (dense) or appended (queue).
template <int IN_REP, int OUT>
__device__ __forceinline__ void bfs_pull_dev(const DevGraph &g, int32_t *depth, int next, const uint8_t *in_bool,
                                             const unsigned long long *in_bits, const OutFrontier &out, Tid t,
                                             long long &ne) {
    // workgroup-uniform iterations (the appends are staged per workgroup, the
    // unfused forms count per lane and add once per workgroup)
    __shared__ StageLDS s_st;
    __shared__ int s_cnt;
    if (threadIdx.x == 0) { s_st.c = 0; s_cnt = 0; }
    __syncthreads();
    int found_cnt = 0;
    const long long stride = (long long)t.nblocks * kBlock;
    for (long long base = (long long)t.block * kBlock; base < g.n; base += stride) {
        const long long v0 = base + threadIdx.x;
        const int v = (int)v0;
        bool found = false;
        if (v < g.n && depth[v] < 0) {
            const int end = g.in_row_ptr[v + 1];
            // parents (in-neighbours) probed kEdgeBatch at a time (their loads
            // overlap); stop at the first parent in the input frontier,
            // counting edges up to it
            for (int e0 = g.in_row_ptr[v]; e0 < end && !found; e0 += kEdgeBatch) {
                int uu[kEdgeBatch];
                bool in[kEdgeBatch];
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) uu[b] = g.in_col[e0 + b < end ? e0 + b : end - 1];
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++)
                    in[b] = IN_REP == kRepBoolmap ? (in_bool[uu[b]] != 0) : bit_test(in_bits, uu[b]);
#pragma unroll
                for (int b = 0; b < kEdgeBatch; b++) {
                    if (!found && e0 + b < end) {
                        ne++;
                        found = in[b];
                    }
                }
            }
            if (found) depth[v] = next;
        }
        if constexpr (OUT == kCreateFused) {
            // the stage holds eight tiles: one flush (one atomic on the queue
            // count) per eight tiles and at the workgroup's last tile
            emit_staged<kCreateFused, kDedupNone>(out, s_st, found, v);
            if ((base / stride) % 8 == 7 || base + stride >= g.n) emit_flush<kCreateFused>(out, s_st);
        } else {
            const uint64_t word = __ballot(found);
            if constexpr (OUT == kCreateBitmap) {
                if (lane_id() == 0 && v0 < ((long long)g.n + 63) / 64 * 64) out.bitmap[v0 >> 6] = word;
            } else {
                if (v < g.n) out.boolmap[v] = found ? 1 : 0;
            }
            found_cnt += found ? 1 : 0;
        }
    }
    if constexpr (OUT != kCreateFused) {
        const int wsum = wave_sum(found_cnt);
        if (lane_id() == 0 && wsum) atomicAdd(&s_cnt, wsum);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomic_add_i32(out.count, s_cnt);
    }
}

template <int IN_REP, int OUT>
__global__ __launch_bounds__(kBlock) void k_bfs_pull(DevGraph g, int32_t *depth, int next, const uint8_t *in_bool,
                                                     const unsigned long long *in_bits, OutFrontier out,
                                                     unsigned long long *ecount) {
    long long ne = 0;
    bfs_pull_dev<IN_REP, OUT>(g, depth, next, in_bool, in_bits, out, Tid::here(), ne);
    flush_edge_count(ne, ecount);
}

// ---- fused (persistent) BFS: the level loop runs on the device -----------------------
// cnt[0..2]: rotating frontier sizes (input of level i is cnt[i % 3]);
// cnt[3]: levels executed, cnt[4]: pull levels, cnt[6]: overflow flag.
struct FusedBfsArgs {
    DevGraph g;
    int32_t *depth;
    int32_t *q0, *q1;
    int32_t *cnt;
    uint8_t *map_bool;
    unsigned long long *map_bits;
    float threshold;
    GridBarrier bar;
    unsigned long long *ecount;
    long long *scan, *scan_part;  // STRICT: the frontier's degree scan and per-workgroup sums
};

// S2: 0 = no pull schedule, 1 = pull over a boolmap, 2 = pull over a bitmap
template <int LB, int S2>
__global__ __launch_bounds__(kBlock) void k_bfs_fused(FusedBfsArgs a) {
    const Tid t = Tid::here();
    const int n = a.g.n;
    long long ne = 0;
    GridBarrier bar = a.bar;
    int32_t *qin = a.q0, *qout = a.q1;
    int it = 0, pulls = 0;
    for (;;) {
        const int cnt = load_relaxed(&a.cnt[it % 3]);
        if (cnt == 0) break;
        if (t.block == 0 && threadIdx.x == 0)
            __hip_atomic_store(&a.cnt[(it + 2) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        OutFrontier o{};
        o.q = qout;
        o.count = &a.cnt[(it + 1) % 3];
        o.cap = n;
        o.overflow = &a.cnt[6];
        const bool pull = S2 != 0 && (double)cnt > (double)a.threshold * (double)n;
        if (!pull) {
            const SrcQueue src{qin, cnt};
            BfsPush f{a.depth, it + 1};
            if constexpr (LB == GG_LB_VERTEX_BASED) lb_vp<kCreateFused, kDedupNone, false>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_WM) lb_wm<kCreateFused, kDedupNone>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_CM) lb_cm<kCreateFused, kDedupNone, false>(a.g, src, f, o, t, ne);
            else if constexpr (LB == GG_LB_STRICT) {
                if (!grid_degree_scan(a.g, src, a.scan, a.scan_part, bar)) break;
                lb_strict<kCreateFused, kDedupNone>(a.g, src, a.scan, f, o, t, ne);
            } else lb_etwc<kCreateFused, kDedupNone, false>(a.g, src, f, o, t, ne);
        } else {
            pulls++;
            // dense input map from the queue: clear, barrier, scatter, barrier
            const long long stride = (long long)t.nblocks * kBlock;
            const long long gid = (long long)t.block * kBlock + threadIdx.x;
            if constexpr (S2 == 1) {
                for (long long i = gid; i < n; i += stride) a.map_bool[i] = 0;
            } else {
                for (long long i = gid; i < (n + 63) / 64; i += stride) a.map_bits[i] = 0ull;
            }
            if (!grid_sync(bar)) break;
            for (long long i = gid; i < cnt; i += stride) {
                const int v = qin[i];
                if constexpr (S2 == 1) a.map_bool[v] = 1;
                else atomic_or_u64(&a.map_bits[v >> 6], 1ull << (v & 63));
            }
            if (!grid_sync(bar)) break;
            if constexpr (S2 == 1)
                bfs_pull_dev<kRepBoolmap, kCreateFused>(a.g, a.depth, it + 1, a.map_bool, nullptr, o, t, ne);
            else
                bfs_pull_dev<kRepBitmap, kCreateFused>(a.g, a.depth, it + 1, nullptr, a.map_bits, o, t, ne);
        }
        if (!grid_sync(bar)) break;
        int32_t *tq = qin; qin = qout; qout = tq;
        it++;
    }
    if (t.block == 0 && threadIdx.x == 0) { a.cnt[3] = it; a.cnt[4] = pulls; }
    flush_edge_count(ne, a.ecount);
}

template <int LB>
static const void *fused_kernel_s2(int s2) {
    if (s2 == 0) return (const void *)k_bfs_fused<LB, 0>;
    if (s2 == 1) return (const void *)k_bfs_fused<LB, 1>;
    return (const void *)k_bfs_fused<LB, 2>;
}

void bfs_fused(Ctx &c, Graph &G, Workspace &ws, int32_t src, const gg_schedule &s, int32_t *depth,
               gg_stats *st) {
    const DevGraph g = G.view();
    const gg_simple_schedule &s1 = s.s1;
    int s2 = 0;
    if (s.hybrid && s.s2.direction == GG_PULL) s2 = s.s2.pull_rep == GG_REP_BITMAP ? 2 : 1;
    const void *kern = nullptr;
    switch (s1.load_balance) {
    case GG_LB_VERTEX_BASED: kern = fused_kernel_s2<GG_LB_VERTEX_BASED>(s2); break;
    case GG_LB_WM: kern = fused_kernel_s2<GG_LB_WM>(s2); break;
    case GG_LB_CM: kern = fused_kernel_s2<GG_LB_CM>(s2); break;
    case GG_LB_ETWC: kern = fused_kernel_s2<GG_LB_ETWC>(s2); break;
    case GG_LB_STRICT: kern = fused_kernel_s2<GG_LB_STRICT>(s2); break;
    default: throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, "kernel fusion supports VERTEX_BASED, WM, CM, ETWC and STRICT");
    }
    const size_t nb = ((size_t)g.n + 255) / 256 * 256;
    ws.q[0].ensure((size_t)g.n);
    ws.q[1].ensure((size_t)g.n);
    ws.counters.ensure(64);
    ws.boolmap[0].ensure(nb);
    ws.bitmap[0].ensure(nb / 64);
    ws.h_i32.ensure(16);
    fill_i32(c, ws.counters.p, 64, 0);
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks_for(g.n, kBlock, 8192)), dim3(kBlock), 0, c.s, depth, g.n, src,
                       ws.q[0].p);
    GG_CHECK_LAUNCH();
    fill_i32(c, ws.counters.p, 1, 1);  // |F0| = 1
    c.launches++;
    const int blocks = fused_grid_for(kern, G, c.num_cus);
    if (s1.load_balance == GG_LB_STRICT) {
        ws.scan.ensure((size_t)g.n + 1);
        ws.scan_part.ensure((size_t)blocks);
    }
    FusedBfsArgs a{g, depth, ws.q[0].p, ws.q[1].p, ws.counters.p, ws.boolmap[0].p, ws.bitmap[0].p,
                   s.threshold, prepare_barrier(c, ws, blocks), c.edge_counter, ws.scan.p, ws.scan_part.p};
    void *args[] = {&a};
    launch_cooperative(c, kern, blocks, args);
    check_barrier(c, ws);
    GG_HIP(hipMemcpyAsync(ws.h_i32.p, ws.counters.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    require(ws.h_i32.p[6] == 0, GG_ERR_OUT_OF_MEMORY, "fused BFS frontier overflow");
    if (st) {
        st->fused = 1;
        st->iterations = ws.h_i32.p[3];
        st->pull_iterations = ws.h_i32.p[4];
        st->push_iterations = st->iterations - st->pull_iterations;
    }
}

template <int IN_REP>
static void launch_pull(Ctx &c, const DevGraph &g, int32_t *depth, int next, const uint8_t *ib,
                        const unsigned long long *it, const OutFrontier &o, int create) {
    // eight tiles per workgroup: every workgroup adds its count (or flushes its
    // appends) with one atomic on a single address, and those serialise
    const dim3 grid(blocks_for(g.n, kBlock * 8, 16384)), block(kBlock);
    if (create == kCreateFused)
        hipLaunchKernelGGL((k_bfs_pull<IN_REP, kCreateFused>), grid, block, 0, c.s, g, depth, next, ib, it, o, c.edge_counter);
    else if (create == kCreateBoolmap)
        hipLaunchKernelGGL((k_bfs_pull<IN_REP, kCreateBoolmap>), grid, block, 0, c.s, g, depth, next, ib, it, o, c.edge_counter);
    else
        hipLaunchKernelGGL((k_bfs_pull<IN_REP, kCreateBitmap>), grid, block, 0, c.s, g, depth, next, ib, it, o, c.edge_counter);
    GG_CHECK_LAUNCH();
    c.launches++;
}

void bfs_pull_step(Ctx &c, const DevGraph &g, FrontierState &fs, const gg_simple_schedule &s, int32_t *depth,
                   int next) {
    const uint8_t *ib = nullptr;
    const unsigned long long *it = nullptr;
    if (s.pull_rep == GG_REP_BITMAP) it = fs.as_bitmap();
    else ib = fs.as_boolmap();
    OutFrontier o{};
    o.overflow = fs.cnt(2);
    o.count = fs.cnt(0);
    fill_i32(c, fs.cnt(0), 1, 0);
    const int create = s.frontier_creation;
    if (create == kCreateFused) { o.q = fs.ws.q[fs.qi ^ 1].p; o.cap = (int32_t)fs.qcap; }
    else if (create == kCreateBoolmap) o.boolmap = fs.ws.boolmap[fs.bi ^ 1].p;
    else o.bitmap = fs.ws.bitmap[fs.ti ^ 1].p;
    if (ib) launch_pull<kRepBoolmap>(c, g, depth, next, ib, it, o, create);
    else launch_pull<kRepBitmap>(c, g, depth, next, ib, it, o, create);
    fs.commit_pull(create);
}

void bfs_run(Graph &G, int32_t src, const gg_schedule &s, int32_t *depth, hipStream_t stream, gg_stats *st) {
    Lease ws(G);
    bfs_run_ws(G, *ws, src, s, depth, stream, st);
}

void bfs_run_ws(Graph &G, Workspace &wsr, int32_t src, const gg_schedule &s, int32_t *depth, hipStream_t stream,
                gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    Workspace *ws = &wsr;
    if (s.s1.load_balance == GG_LB_EDGE_ONLY || (s.hybrid && s.s2.load_balance == GG_LB_EDGE_ONLY))
        ensure_coo(c, G);
    if (schedule_pulls(s)) ensure_transpose(c, G);  // directed graphs: PULL reads in-edges
    const DevGraph g = G.view();
    if (s.s1.kernel_fusion) {
        bfs_fused(c, G, *ws, src, s, depth, st);
        scope.finish();
        return;
    }
    FrontierState fs(c, *ws, g.n, g.n);
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks_for(g.n, kBlock, 8192)), dim3(kBlock), 0, c.s, depth, g.n, src,
                       fs.queue());
    GG_CHECK_LAUNCH();
    c.launches++;
    fs.count = 1;
    int level = 0;
    while (fs.count > 0) {
        const gg_simple_schedule &sc = pick(s, fs.count, g.n);
        if (st) st->vertices_processed += fs.count;
        if (sc.direction == GG_PUSH) {
            const int32_t *q = fs.as_queue();
            // the CAS hands each vertex to one edge per round, so the output
            // queue holds no duplicates for deduplication to remove (as in the
            // fused kernel and BC's push)
            const int dd = kDedupNone;
            OutFrontier o = fs.prep_out(sc.frontier_creation, dd, level + 1, sc.load_balance);
            PushPlan p{sc.load_balance, sc.frontier_creation, dd};
            push_apply(c, g, *ws, p, q, fs.count, BfsPush{depth, level + 1}, o, member_map(*ws, g.n, p.lb));
            fs.commit(sc.frontier_creation);
            if (st) st->push_iterations++;
        } else {
            bfs_pull_step(c, g, fs, sc, depth, level + 1);
            if (st) st->pull_iterations++;
        }
        level++;
        if (st) st->iterations++;
    }
    scope.finish();
}

}  // namespace gg
