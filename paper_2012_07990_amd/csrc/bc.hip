// Single-source betweenness (Brandes) on the frontier-driven traversal. The
// paper evaluates BC with the direction-optimising hybrid schedule
// (Evaluation section, "Algorithms" and "BC").
//
// Forward: level-synchronous BFS that also counts shortest paths. PUSH claims
// unvisited neighbours with a compare-and-swap of the level (as BFS) and adds
// sigma(u) to sigma(v) for every v one level deeper; PULL lets each unvisited
// vertex sum sigma over all its parents in the input frontier (no early
// exit: every parent contributes). sigma is uint64; a wrapping add raises the
// overflow flag. The frontiers are stored back to back in one array, so the
// vertices of each level stay available for the backward pass.
// Backward: from the deepest level up, each vertex v pulls
//   delta(v) = sum_{w in N(v), depth(w) = depth(v)+1} sigma(v)/sigma(w) * (1 + delta(w))
// with FP64 arithmetic in an order fixed by v's degree alone (deterministic,
// so batched and single-source runs give identical bits); delta(src) = 0.
#include "algos.hpp"
#include "bc.hpp"
#include "driver.hpp"

namespace gg {

struct BcPush {
    int32_t *depth;
    unsigned long long *sigma;
    int next;
    int32_t *ovf;
    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    using Pre = int;
    __device__ __forceinline__ Pre load(int, int v, int) const { return depth[v]; }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, load(u, v, e)); }
    __device__ __forceinline__ int apply(int u, int v, int, Pre dv) const {
        int d = dv;
        bool claimed = false;
        if (d < 0) {
            d = atomic_cas_i32(&depth[v], -1, next);
            if (d == -1) { claimed = true; d = next; }
        }
        if (d == next) {
            const unsigned long long su = sigma[u];
            const unsigned long long old = atomic_add_u64(&sigma[v], su);
            if (old + su < old) *ovf = 1;
        }
        return claimed ? v : -1;
    }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};

__global__ __launch_bounds__(kBlock) void k_bc_init(int32_t *depth, unsigned long long *sigma, double *delta, int n,
                                                    int src, int32_t *order) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        depth[v] = v == src ? 0 : -1;
        sigma[v] = v == src ? 1ull : 0ull;
        delta[v] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) order[0] = src;
}

// PULL forward step: every unvisited v sums sigma over all its neighbours in
// the level-L frontier (probed in a boolmap or bitmap). Integer sums are
// order-free, so the lanes of a workgroup share the work ETWC-style: a
// vertex's neighbours are scanned by one lane (degree < 64), a wavefront or
// the whole workgroup, with an atomic add of the partial sums.
// butterfly sum over the wave that reports any wrapping add (all terms are
// non-negative, so the total fits iff no partial sum wraps)
__device__ __forceinline__ unsigned long long wave_sum_checked(unsigned long long x, bool &wrap) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long y = __shfl_xor(x, off, kWave);
        wrap |= x + y < x;
        x += y;
    }
    return x;
}

template <int REP>
__global__ __launch_bounds__(kBlock) void k_bc_pull(DevGraph g, int32_t *depth, unsigned long long *sigma, int next,
                                                    const uint8_t *in_bool, const unsigned long long *in_bits,
                                                    OutFrontier out, int32_t *ovf, unsigned long long *ecount) {
    __shared__ int q_v[2][kBlock];
    __shared__ int q_n[2];
    __shared__ unsigned long long s_sum[kBlock];
    __shared__ int s_any[kBlock];
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    long long ne = 0;
    __shared__ StageLDS s_st;  // the level's queue appends, one global atomic per flush
    auto member = [&](int u) { return REP == kRepBoolmap ? (in_bool[u] != 0) : bit_test(in_bits, u); };
    if (tid == 0) s_st.c = 0;
    __syncthreads();
    for (int base = blockIdx.x * kBlock; base < g.n; base += gridDim.x * kBlock) {
        if (tid < 2) q_n[tid] = 0;
        s_sum[tid] = 0;
        s_any[tid] = 0;
        __syncthreads();
        const int v = base + tid;
        if (v < g.n && depth[v] < 0) {
            const int beg = g.in_row_ptr[v], end = g.in_row_ptr[v + 1];
            const int deg = end - beg;
            if (deg < kWave) {
                unsigned long long s = 0;
                int any = 0;
                for (int e0 = beg; e0 < end; e0 += kEdgeBatch) {  // loads of a batch overlap
                    int uu[kEdgeBatch];
                    bool in[kEdgeBatch];
                    unsigned long long su[kEdgeBatch];
#pragma unroll
                    for (int b = 0; b < kEdgeBatch; b++) uu[b] = g.in_col[e0 + b < end ? e0 + b : end - 1];
#pragma unroll
                    for (int b = 0; b < kEdgeBatch; b++) in[b] = e0 + b < end && member(uu[b]);
#pragma unroll
                    for (int b = 0; b < kEdgeBatch; b++) su[b] = in[b] ? sigma[uu[b]] : 0ull;
#pragma unroll
                    for (int b = 0; b < kEdgeBatch; b++) {
                        if (e0 + b < end) ne++;
                        if (in[b]) {
                            if (s + su[b] < s) *ovf = 1;
                            s += su[b];
                            any = 1;
                        }
                    }
                }
                s_sum[tid] = s;
                s_any[tid] = any;
            } else {
                const int k = atomicAdd(&q_n[deg < kBlock * 16 ? 0 : 1], 1);
                q_v[deg < kBlock * 16 ? 0 : 1][k] = tid;
            }
        }
        __syncthreads();
        for (int k = wib; k < q_n[0]; k += kBlock / kWave) {
            const int slot = q_v[0][k], vv = base + slot;
            unsigned long long s = 0;
            int any = 0;
            bool wrap = false;
            for (int e = g.in_row_ptr[vv] + lane; e < g.in_row_ptr[vv + 1]; e += kWave) {
                const int u = g.in_col[e];
                ne++;
                if (member(u)) {
                    const unsigned long long su = sigma[u];
                    wrap |= s + su < s;
                    s += su;
                    any = 1;
                }
            }
            s = wave_sum_checked(s, wrap);
            any = __any(any);
            if (__any(wrap) && lane == 0) *ovf = 1;
            if (lane == 0) { s_sum[slot] = s; s_any[slot] = any; }
        }
        for (int k = 0; k < q_n[1]; k++) {
            const int slot = q_v[1][k], vv = base + slot;
            unsigned long long s = 0;
            int any = 0;
            bool wrap = false;
            for (int e = g.in_row_ptr[vv] + tid; e < g.in_row_ptr[vv + 1]; e += kBlock) {
                const int u = g.in_col[e];
                ne++;
                if (member(u)) {
                    const unsigned long long su = sigma[u];
                    wrap |= s + su < s;
                    s += su;
                    any = 1;
                }
            }
            s = wave_sum_checked(s, wrap);
            any = __any(any);
            if (__any(wrap) && lane == 0) *ovf = 1;
            if (lane == 0 && any) {
                const unsigned long long old = atomicAdd(&s_sum[slot], s);
                if (old + s < old) *ovf = 1;
                s_any[slot] = 1;
            }
        }
        __syncthreads();
        bool found = false;
        if (v < g.n && s_any[tid]) {
            found = true;
            depth[v] = next;
            sigma[v] = s_sum[tid];
        }
        emit_staged<kCreateFused, kDedupNone>(out, s_st, found, v);
        // one flush (one atomic on the level's count) per eight tiles
        if ((base / (gridDim.x * kBlock)) % 8 == 7 || base + gridDim.x * kBlock >= g.n)
            emit_flush<kCreateFused>(out, s_st);
    }
    flush_edge_count(ne, ecount);
}

// Backward step over the vertices of one level. The summation order of a
// vertex depends only on its degree (never on the schedule): degree < 64 is
// summed by one lane in CSR order; 64 <= degree < 4096 by one wavefront (lane
// j sums neighbours j, j+64, ... in order, then a fixed butterfly); larger by
// the whole workgroup (lane-strided partials, butterfly per wave, waves in
// order). The multi-source pass uses the same rule, so results are bitwise
// identical between single and batched runs.

// The sum of t(w) over the successors w among edges e0, e0 + stride, ...
// below e_end, in that order, with the loads of kEdgeBatch edges issued
// before their additions (the order of the additions, and so the rounding, is
// the plain loop's). DT: the depth array read for the successor test (one
// byte per vertex when the levels fit, so the array stays in L2).
template <class DT>
__device__ __forceinline__ double bc_terms(const DevGraph &g, int e0, int e_end, int stride, DT dv1,
                                           const DT *depth, const double *tv, double acc) {
    for (int e = e0; e < e_end; e += kEdgeBatch * stride) {
        int ww[kEdgeBatch];
        DT dd[kEdgeBatch];
        double tt[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) {
            const int eb = e + b * stride;
            ww[b] = g.col[eb < e_end ? eb : e];
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) dd[b] = depth[ww[b]];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++) {
            const bool on = e + b * stride < e_end && dd[b] == dv1;
            tt[b] = on ? tv[ww[b]] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; b++)
            if (e + b * stride < e_end && dd[b] == dv1) acc = acc + tt[b];
    }
    return acc;
}

__device__ __forceinline__ void bc_set(double *delta, double *tv, int v, double sv, double sum_t) {
    const double d = bc_delta(sv, sum_t);
    delta[v] = d;
    tv[v] = bc_tval(sv, d);
}

// the vertices of level L (ids in level_ids); dv1 = L + 1 in the type of dep
template <class DT>
__global__ __launch_bounds__(kBlock) void k_bc_backward(DevGraph g, const int32_t *level_ids, int count,
                                                        const DT *dep, DT dv1, const unsigned long long *sigma,
                                                        double *delta, double *tv, int src) {
    __shared__ int q_v[2][kBlock];
    __shared__ int q_n[2];
    __shared__ double s_w[kBlock / kWave];
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    for (int base = blockIdx.x * kBlock; base < count; base += gridDim.x * kBlock) {
        if (tid < 2) q_n[tid] = 0;
        __syncthreads();
        const int i = base + tid;
        if (i < count) {
            const int v = level_ids[i];
            const int deg = g.row_ptr[v + 1] - g.row_ptr[v];
            if (v == src) {
                delta[v] = 0.0;
            } else if (deg < kBcWaveDeg) {
                const double sum_t = bc_terms(g, g.row_ptr[v], g.row_ptr[v + 1], 1, dv1, dep, tv, 0.0);
                bc_set(delta, tv, v, (double)sigma[v], sum_t);
            } else {
                const int k = atomicAdd(&q_n[deg < kBcBlockDeg ? 0 : 1], 1);
                q_v[deg < kBcBlockDeg ? 0 : 1][k] = v;
            }
        }
        __syncthreads();
        for (int k = wib; k < q_n[0]; k += kBlock / kWave) {
            const int v = q_v[0][k];
            double acc = bc_terms(g, g.row_ptr[v] + lane, g.row_ptr[v + 1], kWave, dv1, dep, tv, 0.0);
            acc = wave_sum(acc);
            if (lane == 0) bc_set(delta, tv, v, (double)sigma[v], acc);
        }
        for (int k = 0; k < q_n[1]; k++) {
            const int v = q_v[1][k];
            double acc = bc_terms(g, g.row_ptr[v] + tid, g.row_ptr[v + 1], kBlock, dv1, dep, tv, 0.0);
            acc = wave_sum(acc);
            __syncthreads();
            if (lane == 0) s_w[wib] = acc;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int w = 0; w < kBlock / kWave; w++) t += s_w[w];
                bc_set(delta, tv, v, (double)sigma[v], t);
            }
        }
        __syncthreads();
    }
}

// one-byte copy of the BFS depths (255 = unreached) when every level fits
__global__ __launch_bounds__(kBlock) void k_depth8(const int32_t *depth, int n, uint8_t *d8) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int d = depth[v];
        d8[v] = d < 0 ? (uint8_t)255 : (uint8_t)d;
    }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double *in, float *out, int n) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) out[v] = (float)in[v];
}

void bc_run(Graph &G, int32_t src, const gg_schedule &sch, uint64_t *sigma_out, float *delta_out, hipStream_t stream,
            gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    Lease ws(G);
    if (sch.s1.load_balance == GG_LB_EDGE_ONLY || (sch.hybrid && sch.s2.load_balance == GG_LB_EDGE_ONLY))
        ensure_coo(c, G);
    if (schedule_pulls(sch)) ensure_transpose(c, G);  // directed graphs: PULL sums over in-edges
    const DevGraph g = G.view();
    const int n = g.n;
    unsigned long long *sigma = reinterpret_cast<unsigned long long *>(sigma_out);
    const size_t nb = ((size_t)n + 255) / 256 * 256;
    ws->q[0].ensure(n);  // all frontiers back to back (level order)
    ws->counters.ensure(64);
    ws->boolmap[0].ensure(nb);
    ws->bitmap[0].ensure(nb / 64);
    ws->aux_i32[3].ensure(n);  // depth
    ws->aux_f64[0].ensure(n);  // delta (fp64)
    ws->aux_f64[1].ensure(n);  // t = (1 + delta) / sigma, written with delta
    ws->h_i32.ensure(16);
    int32_t *order = ws->q[0].p, *depth = ws->aux_i32[3].p, *ctr = ws->counters.p;
    double *delta = ws->aux_f64[0].p, *tv = ws->aux_f64[1].p;
    fill_i32(c, ctr, 64, 0);
    hipLaunchKernelGGL(k_bc_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, depth, sigma, delta, n,
                       src, order);
    GG_CHECK_LAUNCH();
    c.launches++;
    std::vector<int> off{0, 1};  // level L occupies order[off[L], off[L+1])
    for (int L = 0;; L++) {
        const int cnt = off[L + 1] - off[L];
        if (cnt == 0) break;
        const gg_simple_schedule &sc = pick(sch, cnt, n);
        OutFrontier o{};
        o.q = order + off[L + 1];
        o.cap = n - off[L + 1];
        o.count = ctr + 0;
        o.overflow = ctr + 2;
        // a STRICT push clears the level's count in its degree scan
        if (sc.direction == GG_PUSH && sc.load_balance == GG_LB_STRICT) o.clear = ctr;
        else fill_i32(c, ctr, 1, 0);
        if (st) { st->iterations++; st->vertices_processed += cnt; }
        if (sc.direction == GG_PUSH) {
            push_apply(c, g, *ws, PushPlan{sc.load_balance, kCreateFused, kDedupNone}, order + off[L], cnt,
                       BcPush{depth, sigma, L + 1, ctr + 3}, o, member_map(*ws, n, sc.load_balance));
            if (st) st->push_iterations++;
        } else {
            const unsigned long long *ib = nullptr;
            const uint8_t *bb = nullptr;
            if (sc.pull_rep == GG_REP_BITMAP) {
                fill_u64(c, ws->bitmap[0].p, (long long)nb / 64, 0);
                queue_to_bitmap(c, order + off[L], cnt, ws->bitmap[0].p);
                ib = ws->bitmap[0].p;
            } else {
                fill_u8(c, ws->boolmap[0].p, (long long)nb, 0);
                queue_to_boolmap(c, order + off[L], cnt, ws->boolmap[0].p);
                bb = ws->boolmap[0].p;
            }
            const dim3 grid(blocks_for(n, kBlock * 8, 16384));  // eight tiles per workgroup
            if (bb)
                hipLaunchKernelGGL(k_bc_pull<kRepBoolmap>, grid, dim3(kBlock), 0, c.s, g, depth, sigma, L + 1, bb, ib,
                                   o, ctr + 3, c.edge_counter);
            else
                hipLaunchKernelGGL(k_bc_pull<kRepBitmap>, grid, dim3(kBlock), 0, c.s, g, depth, sigma, L + 1, bb, ib,
                                   o, ctr + 3, c.edge_counter);
            GG_CHECK_LAUNCH();
            c.launches++;
            if (st) st->pull_iterations++;
        }
        const int nxt = read_i32(c, ctr, ws->h_i32.p);
        off.push_back(off[L + 1] + nxt);
    }
    GG_HIP(hipMemcpyAsync(ws->h_i32.p, ctr, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    require(ws->h_i32.p[2] == 0, GG_ERR_OUT_OF_MEMORY, "BC frontier overflow");
    require(ws->h_i32.p[3] == 0, GG_ERR_OVERFLOW, "a shortest-path count exceeds 2^64-1");
    // backward, deepest level first
    const int levels = (int)off.size() - 2;
    const bool small = levels < 255;  // depths 0..254 fit a byte next to the 255 marker
    uint8_t *d8 = ws->boolmap[0].p;   // free after the forward pass (nb >= n bytes)
    if (small) {
        hipLaunchKernelGGL(k_depth8, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, depth, n, d8);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
    // from the deepest level (no successors: delta 0, t = 1/sigma) up
    for (int L = levels - 1; L >= 0; L--) {
        const int cnt = off[L + 1] - off[L];
        if (small)
            hipLaunchKernelGGL(k_bc_backward<uint8_t>, dim3(blocks_for(cnt, kBlock, 16384)), dim3(kBlock), 0, c.s, g,
                               order + off[L], cnt, (const uint8_t *)d8, (uint8_t)(L + 1), sigma, delta, tv, src);
        else
            hipLaunchKernelGGL(k_bc_backward<int32_t>, dim3(blocks_for(cnt, kBlock, 16384)), dim3(kBlock), 0, c.s, g,
                               order + off[L], cnt, (const int32_t *)depth, (int32_t)(L + 1), sigma, delta, tv, src);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, delta, delta_out, n);
    GG_CHECK_LAUNCH();
    c.launches++;
    GG_HIP(hipStreamSynchronize(c.s));
    scope.finish();
}

}  // namespace gg
