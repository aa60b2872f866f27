// Runtime support for programs compiled from the algorithm and scheduling
// languages (the compiler in paper_2012_07990_amd/compiler): generated code
// defines its edge and vertex functors and a main function, and calls these
// templates for the operators. A generated module is compiled against these
// headers and linked with libgg.so (frontier conversions, scans, fills).
//
// Edge functors follow the load balancers' interface (lb.hpp): active(x),
// done(x), load / apply / edge, begin / flush. A PUSH step runs through
// push_apply with the schedule's load balance, frontier creation and
// deduplication; a PULL step runs k_gen_pull, one lane per destination that
// passes the `to` filter, over its in-neighbours in the input frontier, and
// stops at the first one after which the filter fails (the early exit the
// GPU Backend section describes for pull traversals).
//
// A while-loop scheduled with kernel fusion runs as one persistent
// cooperative launch (k_gen_fused): the loop state (frontier sizes, the two
// queues, the round counter) lives in device memory, each round's operator
// runs as the grid-stride __device__ form of its load balancer, and rounds
// are separated by the grid barrier of fused.hpp.
#pragma once

#include <climits>

#include "algos.hpp"
#include "driver.hpp"
#include "fused.hpp"
#include "handles.hpp"

namespace gg {
namespace gen {

// PULL edgeset.apply (from a dense frontier, or every vertex when ALL) over
// the grid described by t: one lane per destination
template <int IN_REP, int CREATE, bool ALL, class F>
__device__ void gen_pull_dev(const DevGraph &g, F &f, const uint8_t *in_bool, const unsigned long long *in_bits,
                             const OutFrontier &out, Tid t) {
    __shared__ StageLDS s_st;
    if (threadIdx.x == 0) s_st.c = 0;
    __syncthreads();
    const long long stride = (long long)t.nblocks * kBlock;
    for (long long base = (long long)t.block * kBlock; base < g.n; base += stride) {
        const long long v0 = base + threadIdx.x;
        const int v = (int)v0;
        bool modified = false;
        if (v < g.n && f.active(v)) {
            for (int e = g.in_row_ptr[v]; e < g.in_row_ptr[v + 1]; e++) {
                const int u = g.in_col[e];
                bool in = true;
                if constexpr (!ALL) in = IN_REP == kRepBoolmap ? in_bool[u] != 0 : bit_test(in_bits, u);
                if (!in) continue;
                if (f.apply(u, v, e, f.load(u, v, e)) >= 0) modified = true;
                if (f.done(v)) break;
            }
        }
        if constexpr (CREATE == kCreateFused) {
            emit_staged<kCreateFused, kDedupNone>(out, s_st, modified, v);
            if ((base / stride) % 8 == 7 || base + stride >= g.n) emit_flush<kCreateFused>(out, s_st);
        } else if constexpr (CREATE == kCreateBitmap) {
            const uint64_t word = __ballot(modified);
            if (lane_id() == 0 && v0 < ((long long)g.n + 63) / 64 * 64) out.bitmap[v0 >> 6] = word;
        } else {
            if (v < g.n) out.boolmap[v] = modified ? 1 : 0;
        }
    }
}

template <int IN_REP, int CREATE, bool ALL, class F>
__global__ __launch_bounds__(kBlock) void k_gen_pull(DevGraph g, F f, const uint8_t *in_bool,
                                                     const unsigned long long *in_bits, OutFrontier out) {
    gen_pull_dev<IN_REP, CREATE, ALL>(g, f, in_bool, in_bits, out, Tid::here());
}

// vertices.apply(f)
template <class F>
__global__ __launch_bounds__(kBlock) void k_gen_vertices(int n, F f) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) f(v);
}

template <class F>
void vertices_apply(Ctx &c, int n, F f) {
    hipLaunchKernelGGL(k_gen_vertices<F>, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, n, f);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// fill a vector with a value (a vector's initialiser)
template <class T>
__global__ __launch_bounds__(kBlock) void k_gen_fill(T *p, int n, T v) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = v;
}
template <class T>
void fill(Ctx &c, T *p, int n, T v) {
    hipLaunchKernelGGL(k_gen_fill<T>, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, p, n, v);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// out-degrees (edges.getOutDegrees())
template <class T>
__global__ __launch_bounds__(kBlock) void k_gen_outdeg(DevGraph g, T *p) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < g.n; v += gridDim.x * kBlock)
        p[v] = (T)(g.row_ptr[v + 1] - g.row_ptr[v]);
}
template <class T>
void out_degrees(Ctx &c, const DevGraph &g, T *p) {
    hipLaunchKernelGGL(k_gen_outdeg<T>, dim3(blocks_for(g.n, kBlock, 8192)), dim3(kBlock), 0, c.s, g, p);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// one element written from the host (main's `vec[i] = value;`, and
// frontier.addVertex(i)); an index outside [0, n) is refused
template <class T>
void set_one(Ctx &c, T *p, long long n, int64_t i, T v) {
    require(i >= 0 && i < n, GG_ERR_INVALID_ARG, "vertex index out of range");
    GG_HIP(hipMemcpyAsync(p + i, &v, sizeof(T), hipMemcpyHostToDevice, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
}

// frontier.addVertex(v) on the live queue
inline void add_vertex(Ctx &c, FrontierState &fs, int n, int64_t v) {
    require(v >= 0 && v < n, GG_ERR_INVALID_ARG, "vertex index out of range");
    set_one<int32_t>(c, fs.queue(), fs.qcap, fs.count, (int32_t)v);
    fs.count++;
}

// a frontier holding every vertex (new vertexset{Vertex}(vertices.size()))
__global__ __launch_bounds__(kBlock) inline void k_gen_iota(int32_t *q, int n) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) q[v] = v;
}

// edges.from(frontier).to(filter).apply...(f) under a SimpleGPUSchedule
// (the schedule already picked by the hybrid rule); iter numbers the step
// for monotonic deduplication
template <class F>
void frontier_step(Ctx &c, const DevGraph &g, Workspace &ws, FrontierState &fs, const gg_simple_schedule &sc,
                   F f, int iter) {
    if (sc.direction == GG_PUSH) {
        const int32_t *q = fs.as_queue();
        const int dd = dedup_mode(sc);
        OutFrontier o = fs.prep_out(sc.frontier_creation, dd, iter, sc.load_balance);
        const PushPlan p{sc.load_balance, sc.frontier_creation, dd};
        push_apply(c, g, ws, p, q, fs.count, f, o, member_map(ws, g.n, p.lb));
        fs.commit(sc.frontier_creation);
        return;
    }
    const uint8_t *ib = nullptr;
    const unsigned long long *it = nullptr;
    if (sc.pull_rep == GG_REP_BITMAP) it = fs.as_bitmap();
    else ib = fs.as_boolmap();
    OutFrontier o{};
    o.overflow = fs.cnt(2);
    o.count = fs.cnt(0);
    fill_i32(c, fs.cnt(0), 1, 0);
    const int create = sc.frontier_creation;
    if (create == kCreateFused) {
        o.q = fs.ws.q[fs.qi ^ 1].p;
        o.cap = (int32_t)fs.qcap;
    } else if (create == kCreateBoolmap) {
        o.boolmap = fs.ws.boolmap[fs.bi ^ 1].p;
    } else {
        o.bitmap = fs.ws.bitmap[fs.ti ^ 1].p;
    }
    const dim3 grid(blocks_for(g.n, kBlock * 8, 16384)), block(kBlock);
    if (ib) {
        if (create == kCreateFused) hipLaunchKernelGGL((k_gen_pull<kRepBoolmap, kCreateFused, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
        else if (create == kCreateBoolmap) hipLaunchKernelGGL((k_gen_pull<kRepBoolmap, kCreateBoolmap, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
        else hipLaunchKernelGGL((k_gen_pull<kRepBoolmap, kCreateBitmap, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
    } else {
        if (create == kCreateFused) hipLaunchKernelGGL((k_gen_pull<kRepBitmap, kCreateFused, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
        else if (create == kCreateBoolmap) hipLaunchKernelGGL((k_gen_pull<kRepBitmap, kCreateBoolmap, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
        else hipLaunchKernelGGL((k_gen_pull<kRepBitmap, kCreateBitmap, false, F>), grid, block, 0, c.s, g, f, ib, it, o);
    }
    GG_CHECK_LAUNCH();
    c.launches++;
    if (create != kCreateFused) {
        // the dense output's population (a ballot per 64 destinations)
        fill_i32(c, fs.cnt(0), 1, 0);
        if (create == kCreateBoolmap) count_boolmap(c, o.boolmap, g.n, fs.cnt(0));
        else count_bitmap(c, o.bitmap, g.n, fs.cnt(0));
    }
    fs.commit_pull(create);
}

// edges.apply(f) over every edge: PUSH through the schedule's load balancer
// from a frontier of every vertex (ids = 0..n-1), or PULL over every
// destination's in-edges
template <class F>
void all_edges_step(Ctx &c, const DevGraph &g, Workspace &ws, const int32_t *ids, const gg_simple_schedule &sc,
                    F f) {
    if (sc.direction == GG_PUSH) {
        ws.boolmap[1].ensure(((size_t)g.n + 255) / 256 * 256);
        OutFrontier o{};
        o.boolmap = ws.boolmap[1].p;  // nothing is emitted
        const PushPlan p{sc.load_balance, kCreateBoolmap, kDedupNone};
        push_apply(c, g, ws, p, ids, g.n, f, o, member_map(ws, g.n, p.lb));
        return;
    }
    OutFrontier o{};
    ws.boolmap[1].ensure(((size_t)g.n + 255) / 256 * 256);
    o.boolmap = ws.boolmap[1].p;
    hipLaunchKernelGGL((k_gen_pull<kRepBoolmap, kCreateBoolmap, true, F>), dim3(blocks_for(g.n, kBlock * 8, 16384)),
                       dim3(kBlock), 0, c.s, g, f, nullptr, nullptr, o);
    GG_CHECK_LAUNCH();
    c.launches++;
}


// edges.apply(f) under EdgeBlocking (configLoadBalance(EDGE_ONLY, BLOCKED, N)):
// every edge of the EdgeBlocked COO (destination segments of N vertices,
// built once per graph and width), one launch per segment. f reads the
// weights in the blocked order.
template <class F>
__global__ __launch_bounds__(kBlock) void k_gen_edges_blocked(const int32_t *src, const int32_t *dst, long long lo,
                                                              long long hi, F f) {
    for (long long e = lo + (long long)blockIdx.x * kBlock + threadIdx.x; e < hi; e += (long long)gridDim.x * kBlock)
        (void)f.edge(src[e], dst[e], (int)e);
}

template <class F>
void all_edges_blocked(Ctx &c, Graph &G, int32_t N, F f) {
    edgeblock_prepare(c, G, N);
    const EdgeBlocked *eb;
    {
        std::lock_guard<std::mutex> lk(G.mu);
        eb = G.eb.at(N).get();
    }
    f.w = eb->w.p;
    for (size_t sg = 0; sg + 1 < eb->seg_start.size(); sg++) {
        const long long lo = eb->seg_start[sg], hi = eb->seg_start[sg + 1];
        if (hi <= lo) continue;
        hipLaunchKernelGGL(k_gen_edges_blocked<F>, dim3(blocks_for(hi - lo, kBlock, 16384)), dim3(kBlock), 0, c.s,
                           eb->src.p, eb->dst.p, lo, hi, f);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
}

// ---- kernel fusion: the whole frontier loop in one persistent launch ----------

struct GenFusedArgs {
    DevGraph g;
    int32_t *q0, *q1;        // the two queues (q0 holds the first frontier)
    int32_t *cnt;            // [0..2] rotating frontier sizes, [3] rounds, [4] PULL rounds,
                             // [8..10] rotating overflow flags
    int32_t *tags;           // monotonic-counter deduplication
    int32_t iter0;           // the tag of the round before the loop
    int32_t cap;             // queue capacity
    float threshold;         // hybrid: PULL when |F| > threshold * n
    uint8_t *map_bool;       // PULL input frontier, boolmap form
    unsigned long long *map_bits;  // PULL input frontier, bitmap form
    GridBarrier bar;
    long long *scan, *scan_part;   // STRICT: the frontier's degree scan
};

// The steps of a fused loop, for k_gen_fused and for the kernels generated
// for fused loops with more statements than the operator: a round's head
// (exit test, counters), its operator, whole-vertex applies, and its tail
// (grid barrier, queue swap). Every lane of the grid runs every step.
struct FusedLoopState {
    Tid t;
    GridBarrier bar;
    int32_t *qin, *qout;
    int it, pulls;
};

__device__ __forceinline__ FusedLoopState fused_begin(const GenFusedArgs &a) {
    return FusedLoopState{Tid::here(), a.bar, a.q0, a.q1, 0, 0};
}

// The input frontier's size, or -1 when the loop ends: the frontier is empty,
// or the previous round overflowed its queue. A round's overflow flag is read
// at the head of the next round (after the barrier that ends the round that
// raised it), so every workgroup leaves at the same round.
__device__ __forceinline__ int fused_round_head(const GenFusedArgs &a, const FusedLoopState &s) {
    const int it = s.it;
    if (it > 0 && load_relaxed(&a.cnt[8 + (it + 2) % 3]) != 0) return -1;
    const int cnt = load_relaxed(&a.cnt[it % 3]);
    if (cnt == 0) return -1;
    if (s.t.block == 0 && threadIdx.x == 0) {
        __hip_atomic_store(&a.cnt[(it + 2) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.cnt[8 + (it + 1) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return cnt;
}

// LB: the PUSH load balancer; DD: kDedupNone or kDedupMonotonic; S2: 0 = PUSH
// only, 1 / 2 = hybrid with a PULL step over a boolmap / bitmap. The round's
// output goes to s.qout; false when a grid barrier was aborted.
template <int LB, int DD, int S2, class FP, class FL>
__device__ bool fused_step(const GenFusedArgs &a, FP &fp, FL &fl, FusedLoopState &s, int cnt) {
    const int n = a.g.n;
    const Tid t = s.t;
    long long ne = 0;
    OutFrontier o{};
    o.q = s.qout;
    o.count = &a.cnt[(s.it + 1) % 3];
    o.cap = a.cap;
    o.overflow = &a.cnt[8 + s.it % 3];
    const bool pull = S2 != 0 && (double)cnt > (double)a.threshold * (double)n;
    if (!pull) {
        if constexpr (DD == kDedupMonotonic) {
            o.tags = a.tags;
            o.iter = a.iter0 + s.it + 1;
        }
        const SrcQueue src{s.qin, cnt};
        if constexpr (LB == GG_LB_VERTEX_BASED) lb_vp<kCreateFused, DD, false>(a.g, src, fp, o, t, ne);
        else if constexpr (LB == GG_LB_WM) lb_wm<kCreateFused, DD>(a.g, src, fp, o, t, ne);
        else if constexpr (LB == GG_LB_CM) lb_cm<kCreateFused, DD, false>(a.g, src, fp, o, t, ne);
        else if constexpr (LB == GG_LB_STRICT) {
            if (!grid_degree_scan(a.g, src, a.scan, a.scan_part, s.bar)) return false;
            lb_strict<kCreateFused, DD>(a.g, src, a.scan, fp, o, t, ne);
        } else lb_etwc<kCreateFused, DD, false>(a.g, src, fp, o, t, ne);
        return true;
    }
    s.pulls++;
    // dense input map from the queue: clear, barrier, scatter, barrier
    const long long stride = (long long)t.nblocks * kBlock;
    const long long gid = (long long)t.block * kBlock + threadIdx.x;
    if constexpr (S2 == 1) {
        for (long long i = gid; i < n; i += stride) a.map_bool[i] = 0;
    } else {
        for (long long i = gid; i < (n + 63) / 64; i += stride) a.map_bits[i] = 0ull;
    }
    if (!grid_sync(s.bar)) return false;
    for (long long i = gid; i < cnt; i += stride) {
        const int v = s.qin[i];
        if constexpr (S2 == 1) a.map_bool[v] = 1;
        else atomic_or_u64(&a.map_bits[v >> 6], 1ull << (v & 63));
    }
    if (!grid_sync(s.bar)) return false;
    if constexpr (S2 == 1) gen_pull_dev<kRepBoolmap, kCreateFused, false>(a.g, fl, a.map_bool, nullptr, o, t);
    else if constexpr (S2 == 2) gen_pull_dev<kRepBitmap, kCreateFused, false>(a.g, fl, nullptr, a.map_bits, o, t);
    return true;
}

// vertices.apply(f) inside a fused loop (the caller separates it from the
// steps around it with grid barriers)
template <class F>
__device__ __forceinline__ void fused_vertices(int n, const F &f, Tid t) {
    for (long long v = (long long)t.block * kBlock + threadIdx.x; v < n; v += (long long)t.nblocks * kBlock)
        f((int)v);
}

// the barrier that ends a round, then the swap of the queues
__device__ __forceinline__ bool fused_round_tail(FusedLoopState &s) {
    if (!grid_sync(s.bar)) return false;
    int32_t *tq = s.qin;
    s.qin = s.qout;
    s.qout = tq;
    s.it++;
    return true;
}

__device__ __forceinline__ void fused_end(const GenFusedArgs &a, const FusedLoopState &s) {
    if (s.t.block == 0 && threadIdx.x == 0) {
        a.cnt[3] = s.it;
        a.cnt[4] = s.pulls;
    }
}

template <int LB, int DD, int S2, class FP, class FL>
__global__ __launch_bounds__(kBlock) void k_gen_fused(GenFusedArgs a, FP fp, FL fl) {
    FusedLoopState s = fused_begin(a);
    for (;;) {
        const int cnt = fused_round_head(a, s);
        if (cnt < 0) break;
        if (!fused_step<LB, DD, S2>(a, fp, fl, s, cnt)) break;
        if (!fused_round_tail(s)) break;
    }
    fused_end(a, s);
}

// Host side of a fused loop over the live frontier of fs, for the persistent
// kernel kern (which runs the loop): its grid, the loop state in device memory
// (the first frontier's size, zeroed counters, barrier words, STRICT scan
// buffers) and the arguments. The caller launches kern with
// launch_cooperative(c, kern, blocks, ...) and then calls fused_complete.
struct FusedLaunch {
    GenFusedArgs a;
    int blocks;
};

inline FusedLaunch fused_prepare(Ctx &c, Graph &G, const DevGraph &g, Workspace &ws, FrontierState &fs,
                                 float threshold, const void *kern, bool strict, int iter) {
    const int32_t *q0 = fs.as_queue();
    const int blocks = fused_grid_for(kern, G, c.num_cus);
    const long long cap = fs.qcap < 0x7fffffffll ? fs.qcap : 0x7fffffffll;
    if (strict) {
        ws.scan.ensure((size_t)cap + 1);
        ws.scan_part.ensure((size_t)blocks);
    }
    int32_t *cnt = ws.counters.p + 16;  // the step counters of fs stay below
    fill_i32(c, cnt, 16, 0);
    fill_i32(c, cnt, 1, fs.count);
    GenFusedArgs a{g,
                   const_cast<int32_t *>(q0),
                   ws.q[fs.qi ^ 1].p,
                   cnt,
                   ws.tags.p,
                   iter,
                   (int32_t)cap,
                   threshold,
                   ws.boolmap[fs.bi ^ 1].p,
                   ws.bitmap[fs.ti ^ 1].p,
                   prepare_barrier(c, ws, blocks),
                   ws.scan.p,
                   ws.scan_part.p};
    return FusedLaunch{a, blocks};
}

// After the launch: the barrier's abort flag, the overflow flags, the rounds
// run (iter advances by them); leaves fs empty. Throws GG_ERR_OUT_OF_MEMORY
// when a round's output exceeded the queue (deduplication disabled).
inline void fused_complete(Ctx &c, Workspace &ws, FrontierState &fs, int &iter) {
    check_barrier(c, ws);
    int32_t *cnt = ws.counters.p + 16;
    GG_HIP(hipMemcpyAsync(ws.h_i32.p, cnt, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    require(ws.h_i32.p[8] == 0 && ws.h_i32.p[9] == 0 && ws.h_i32.p[10] == 0, GG_ERR_OUT_OF_MEMORY,
            "output frontier exceeded its queue capacity (enable deduplication)");
    iter += ws.h_i32.p[3];
    fs.count = 0;
}

// Run `while (frontier not empty) frontier = step(frontier)` as one launch
// of k_gen_fused from the live frontier of fs.
template <int LB, int DD, int S2, class FP, class FL>
void fused_loop(Ctx &c, Graph &G, const DevGraph &g, Workspace &ws, FrontierState &fs, float threshold, FP fp,
                FL fl, int &iter) {
    static_assert(LB == GG_LB_VERTEX_BASED || LB == GG_LB_WM || LB == GG_LB_CM || LB == GG_LB_STRICT ||
                      LB == GG_LB_ETWC,
                  "a fused loop runs VERTEX_BASED, WM, CM, STRICT or ETWC");
    static_assert(DD == kDedupNone || DD == kDedupMonotonic, "a fused loop deduplicates with monotonic counters");
    if (fs.count == 0) return;
    const void *kern = (const void *)k_gen_fused<LB, DD, S2, FP, FL>;
    FusedLaunch L = fused_prepare(c, G, g, ws, fs, threshold, kern, LB == GG_LB_STRICT, iter);
    void *args[] = {&L.a, &fp, &fl};
    launch_cooperative(c, kern, L.blocks, args);
    fused_complete(c, ws, fs, iter);
}


// ---- priority queue: applyUpdatePriority with configDelta ----------------------
// Buckets of width delta over an int32 priority vector (the delta-stepping
// priority queue that configDelta parameterises). The ready set is the live
// frontier of fs: vertices of the current bucket k whose priority dropped.
// Later buckets wait in a far queue (a vertex enters each far queue
// generation at most once, by a tag); when the ready set runs empty, the
// smallest bucket in the far queue becomes current and its entries move to
// the ready set.
struct PQView {  // what a generated update functor needs on the device
    int32_t *prio;
    long long bucket_end;  // (k + 1) * delta
    int32_t *farq, *farc;  // the far queue being filled and its size
    int32_t far_cap;
    int32_t *far_tag;
    int32_t far_id;
    int32_t *flags;        // [0] a priority past INT32_MAX - 1, [1] far queue overflow
};

// updatePriorityMin(v, nd): lower prio[v] to nd; true when v joins the ready
// set (its new priority is in the current bucket); to_far when it joins the
// far queue. The caller appends to_far lanes with wave_append (every lane that
// runs the update takes part).
__device__ __forceinline__ bool pq_update_min(const PQView &q, int v, long long nd, bool &to_far) {
    to_far = false;
    if (nd > (long long)INT_MAX - 1) {
        q.flags[0] = 1;
        return false;
    }
    if (nd >= q.prio[v]) return false;  // a stale, larger read only costs the atomic
    const int old = atomic_min_i32(&q.prio[v], (int)nd);
    if (nd >= old) return false;
    if (nd < q.bucket_end) return true;
    to_far = q.far_tag[v] < q.far_id && atomic_max_i32(&q.far_tag[v], q.far_id) < q.far_id;
    return false;
}

// smallest bucket beyond k among the far entries (one atomic per workgroup,
// read first)
__global__ __launch_bounds__(kBlock) inline void k_pq_far_min(const int32_t *farq, const int32_t *fc,
                                                               const int32_t *prio, int delta, int k, int32_t *kmin) {
    __shared__ int s_m[kBlock / kWave];
    const int n = *fc;
    int local = INT_MAX;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int b = prio[farq[i]] / delta;
        if (b > k && b < local) local = b;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int o = __shfl_xor(local, off, kWave);
        local = o < local ? o : local;
    }
    if (lane_id() == 0) s_m[threadIdx.x / kWave] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = INT_MAX;
        for (int w = 0; w < kBlock / kWave; w++) m = s_m[w] < m ? s_m[w] : m;
        if (m != INT_MAX && m < load_relaxed(kmin)) atomic_min_i32(kmin, m);
    }
}

// far entries of bucket knew -> the ready set (deduplicated by the tags of
// `near`); entries of later buckets -> the next far queue generation
__global__ __launch_bounds__(kBlock) inline void k_pq_far_split(const int32_t *farq, const int32_t *fc,
                                                                 const int32_t *prio, int delta, int knew,
                                                                 OutFrontier near, int32_t *nfarq, int32_t *nfarc,
                                                                 int far_cap, int32_t *far_tag, int far_id,
                                                                 int32_t *flags) {
    const int n = *fc;
    const int stride = gridDim.x * kBlock;
    const int iters = (n + stride - 1) / stride;
    for (int it = 0; it < iters; it++) {  // wave-uniform trip count for the appends
        const int i = it * stride + blockIdx.x * kBlock + threadIdx.x;
        bool to_near = false, to_far = false;
        int v = 0;
        if (i < n) {
            v = farq[i];
            const int b = prio[v] / delta;
            if (b == knew) to_near = dedup_first<kDedupMonotonic>(near, v);
            else if (b > knew) to_far = far_tag[v] < far_id && atomic_max_i32(&far_tag[v], far_id) < far_id;
        }
        wave_append(near.q, near.count, near.cap, near.overflow, to_near, v);
        wave_append(nfarq, nfarc, far_cap, flags + 1, to_far, v);
    }
}

struct PQState {
    int32_t *prio = nullptr;
    int64_t start = -1;
    int n = 0;
    int delta = 1;
    int k = 0;   // current bucket
    int fe = 0;  // far queue generation being filled
    int32_t *farq[2] = {nullptr, nullptr};
    int32_t *ctr = nullptr;  // [0..1] far sizes, [2] bucket minimum, [4..5] flags
    int32_t *tags = nullptr;
};

// `pq = new priority_queue(prio, start)` then the loop's first round: the
// ready set holds start, the current bucket is prio[start] / delta
inline void pq_start(Ctx &c, Workspace &ws, FrontierState &fs, PQState &pq, int delta) {
    require(pq.prio != nullptr, GG_ERR_INVALID_ARG, "the priority queue was not created");
    require(pq.start >= 0 && pq.start < pq.n, GG_ERR_INVALID_ARG, "vertex index out of range");
    require(delta >= 1, GG_ERR_INVALID_ARG, "delta must be >= 1");
    pq.delta = delta;
    for (int i = 0; i < 3; i++) ws.aux_i32[i].ensure((size_t)pq.n);
    pq.farq[0] = ws.aux_i32[0].p;
    pq.farq[1] = ws.aux_i32[1].p;
    pq.tags = ws.aux_i32[2].p;
    fill_i32(c, pq.tags, pq.n, 0);
    pq.ctr = ws.counters.p + 40;
    fill_i32(c, pq.ctr, 8, 0);
    const int p0 = read_i32(c, pq.prio + pq.start, ws.h_i32.p);
    require(p0 != INT_MAX, GG_ERR_INVALID_ARG, "the start vertex has no priority");
    pq.k = p0 / delta;
    pq.fe = 0;
    fs.count = 0;
    add_vertex(c, fs, pq.n, pq.start);
}

inline PQView pq_view(const PQState &pq) {
    return PQView{pq.prio, (long long)(pq.k + 1) * pq.delta, pq.farq[pq.fe & 1], pq.ctr + (pq.fe & 1), pq.n,
                  pq.tags, pq.fe + 1, pq.ctr + 4};
}

// `while (pq.finished() == false)` with `frontier = pq.dequeue_ready_set()`:
// true while a ready set is left (fs holds it); an empty ready set advances
// to the smallest bucket in the far queue
inline bool pq_next(Ctx &c, Workspace &ws, FrontierState &fs, PQState &pq, int &iter) {
    for (;;) {
        if (fs.count > 0) return true;
        GG_HIP(hipMemcpyAsync(ws.h_i32.p, pq.ctr, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
        GG_HIP(hipStreamSynchronize(c.s));
        require(ws.h_i32.p[4] == 0, GG_ERR_OVERFLOW, "a priority exceeds INT32_MAX-1");
        require(ws.h_i32.p[5] == 0, GG_ERR_OUT_OF_MEMORY, "far queue overflow");
        const int fc = ws.h_i32.p[pq.fe & 1];
        if (fc == 0) return false;
        fill_i32(c, pq.ctr + 2, 1, INT_MAX);
        hipLaunchKernelGGL(k_pq_far_min, dim3(blocks_for(fc, kBlock * 4, 1024)), dim3(kBlock), 0, c.s,
                           pq.farq[pq.fe & 1], pq.ctr + (pq.fe & 1), pq.prio, pq.delta, pq.k, pq.ctr + 2);
        GG_CHECK_LAUNCH();
        const int knew = read_i32(c, pq.ctr + 2, ws.h_i32.p + 8);
        if (knew == INT_MAX) return false;
        fill_i32(c, pq.ctr + ((pq.fe + 1) & 1), 1, 0);
        OutFrontier o = fs.prep_out(kCreateFused, kDedupMonotonic, iter++);
        hipLaunchKernelGGL(k_pq_far_split, dim3(blocks_for(fc, kBlock, 1024)), dim3(kBlock), 0, c.s,
                           pq.farq[pq.fe & 1], pq.ctr + (pq.fe & 1), pq.prio, pq.delta, knew, o,
                           pq.farq[(pq.fe + 1) & 1], pq.ctr + ((pq.fe + 1) & 1), pq.n, pq.tags, pq.fe + 2,
                           pq.ctr + 4);
        GG_CHECK_LAUNCH();
        c.launches += 2;
        fs.commit(kCreateFused);
        pq.fe++;
        pq.k = knew;
    }
}

}  // namespace gen
}  // namespace gg
