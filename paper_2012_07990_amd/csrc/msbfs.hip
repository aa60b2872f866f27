// Batched multi-source BFS and BC: up to 64 sources share one level-
// synchronous traversal with bit-packed frontiers (bit j of a vertex's word
// is source j), so each edge's column and frontier word are read once for
// all sources.
//
// Per vertex: visited (sources that reached it), front (sources that reached
// it at the current level), next. A level is a PULL sweep: every vertex
// still missing some sources ORs its neighbours' front words, keeps the new
// bits, records their level and (BC) adds each new source's path counts
// sigma_j(u) over the parents u with bit j in front. Per-vertex state is
// stored vertex-major (the K values of a vertex share a cache line) and
// transposed into the k x n row-major outputs at the end.
//
// BC runs the backward pass level by level for all sources at once; every
// (source, vertex) dependency is summed in exactly the order of the single-
// source pass (same degree tiers, same lane striding, same butterflies, the
// same non-contracted step), so batched results equal k single calls bit
// for bit.
#include "algos.hpp"
#include "bc.hpp"
#include "driver.hpp"
#include "fused.hpp"
#include "ms.hpp"

namespace gg {

using u64 = unsigned long long;

__global__ __launch_bounds__(kBlock) void k_ms_init(int n, int K, const int32_t *srcs, u64 *visited, u64 *front,
                                                    int32_t *depth_vm, u64 *sigma_vm, double *delta_vm) {
    __shared__ int s_src[64];
    if (threadIdx.x < 64) s_src[threadIdx.x] = threadIdx.x < K ? srcs[threadIdx.x] : -1;
    __syncthreads();
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        u64 mask = 0;
        for (int j = 0; j < K; j++)
            if (s_src[j] == v) mask |= 1ull << j;
        visited[v] = mask;
        front[v] = mask;
        for (int j = 0; j < K; j++) {
            const bool on = (mask >> j) & 1ull;
            depth_vm[(size_t)v * K + j] = on ? 0 : -1;
            if (sigma_vm) {
                sigma_vm[(size_t)v * K + j] = on ? 1ull : 0ull;
                delta_vm[(size_t)v * K + j] = 0.0;
            }
        }
    }
}

__device__ __forceinline__ u64 wave_or(u64 x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x |= __shfl_xor(x, off, kWave);
    return x;
}

// record the level of the new sources of v
__device__ __forceinline__ void ms_record(int32_t *depth_vm, int K, int v, u64 nb, int level) {
    while (nb) {
        const int j = __ffsll(nb) - 1;
        depth_vm[(size_t)v * K + j] = level;
        nb &= nb - 1;
    }
}

// ---- multi-source BFS level (PULL with early exit once every missing source is found)
__device__ __forceinline__ void msbfs_level(const DevGraph &g, int K, u64 all, u64 *visited, const u64 *front,
                                            u64 *next, int32_t *depth_vm, int level, int32_t *any, Tid t) {
    __shared__ int q_v[kBlock];
    __shared__ int q_n;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    bool found_any = false;
    for (int base = t.block * kBlock; base < g.n; base += t.nblocks * kBlock) {
        if (tid == 0) q_n = 0;
        __syncthreads();
        const int v = base + tid;
        if (v < g.n) {
            const u64 need = all & ~visited[v];
            const int beg = g.row_ptr[v], end = g.row_ptr[v + 1];
            if (need == 0 || end == beg) {
                next[v] = 0;
            } else if (end - beg < kWave) {
                u64 acc = 0;
                for (int e = beg; e < end; e++) {
                    acc |= front[g.col[e]];
                    if ((acc & need) == need) break;
                }
                const u64 nb = acc & need;
                next[v] = nb;
                if (nb) {
                    visited[v] |= nb;
                    ms_record(depth_vm, K, v, nb, level);
                    found_any = true;
                }
            } else {
                q_v[atomicAdd(&q_n, 1)] = v;
            }
        }
        __syncthreads();
        for (int k = wib; k < q_n; k += kBlock / kWave) {
            const int vv = q_v[k];
            const u64 need = all & ~visited[vv];
            u64 acc = 0;
            for (int e = g.row_ptr[vv] + lane; e < g.row_ptr[vv + 1]; e += kWave) acc |= front[g.col[e]];
            acc = wave_or(acc);
            const u64 nb = acc & need;
            if (lane == 0) {
                next[vv] = nb;
                if (nb) {
                    visited[vv] |= nb;
                    ms_record(depth_vm, K, vv, nb, level);
                    found_any = true;
                }
            }
        }
        __syncthreads();
    }
    if (__any(found_any) && lane_id() == 0) *any = 1;
}

// ---- multi-source BC forward level: new sources and their path counts -----------------
constexpr int kBcGroup = 16;  // sources per BC pass (sigma / delta of a vertex: 128 B)

__device__ __forceinline__ void msbc_level(const DevGraph &g, int K, u64 all, u64 *visited, const u64 *front,
                                           u64 *next, int32_t *depth_vm, u64 *sigma_vm, int level, int32_t *any,
                                           int32_t *overflow, Tid t) {
    __shared__ int q_v[kBlock];
    __shared__ int q_n;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    bool found_any = false, wrap = false;
    for (int base = t.block * kBlock; base < g.n; base += t.nblocks * kBlock) {
        if (tid == 0) q_n = 0;
        __syncthreads();
        const int v = base + tid;
        if (v < g.n) {
            const u64 need = all & ~visited[v];
            const int beg = g.row_ptr[v], end = g.row_ptr[v + 1];
            if (need == 0 || end == beg) {
                next[v] = 0;
            } else if (end - beg < kWave) {
                u64 acc = 0, sacc[kBcGroup];
#pragma unroll
                for (int j = 0; j < kBcGroup; j++) sacc[j] = 0;
                for (int e = beg; e < end; e++) {
                    const int u = g.col[e];
                    const u64 f = front[u] & need;
                    if (!f) continue;
                    acc |= f;
#pragma unroll
                    for (int j = 0; j < kBcGroup; j++)
                        if ((f >> j) & 1ull) {
                            const u64 su = sigma_vm[(size_t)u * K + j];
                            wrap |= sacc[j] + su < sacc[j];
                            sacc[j] += su;
                        }
                }
                next[v] = acc;
                if (acc) {
                    visited[v] |= acc;
                    ms_record(depth_vm, K, v, acc, level);
#pragma unroll
                    for (int j = 0; j < kBcGroup; j++)
                        if ((acc >> j) & 1ull) sigma_vm[(size_t)v * K + j] = sacc[j];
                    found_any = true;
                }
            } else {
                q_v[atomicAdd(&q_n, 1)] = v;
            }
        }
        __syncthreads();
        for (int k = wib; k < q_n; k += kBlock / kWave) {
            const int vv = q_v[k];
            const u64 need = all & ~visited[vv];
            u64 acc = 0, sacc[kBcGroup];
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) sacc[j] = 0;
            for (int e = g.row_ptr[vv] + lane; e < g.row_ptr[vv + 1]; e += kWave) {
                const int u = g.col[e];
                const u64 f = front[u] & need;
                if (!f) continue;
                acc |= f;
#pragma unroll
                for (int j = 0; j < kBcGroup; j++)
                    if ((f >> j) & 1ull) {
                        const u64 su = sigma_vm[(size_t)u * K + j];
                        wrap |= sacc[j] + su < sacc[j];
                        sacc[j] += su;
                    }
            }
            acc = wave_or(acc);
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) {
#pragma unroll
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    const u64 y = __shfl_xor(sacc[j], off, kWave);
                    wrap |= sacc[j] + y < sacc[j];
                    sacc[j] += y;
                }
            }
            if (lane == 0) {
                next[vv] = acc;
                if (acc) {
                    visited[vv] |= acc;
                    ms_record(depth_vm, K, vv, acc, level);
#pragma unroll
                    for (int j = 0; j < kBcGroup; j++)
                        if ((acc >> j) & 1ull) sigma_vm[(size_t)vv * K + j] = sacc[j];
                    found_any = true;
                }
            }
        }
        __syncthreads();
    }
    if (__any(found_any) && lane_id() == 0) *any = 1;
    if (__any(wrap) && lane_id() == 0) *overflow = 1;
}

// ---- multi-source BC backward level (same summation order as the single pass) -----------
__device__ __forceinline__ void ms_bc_set(double *delta_vm, double *t_vm, size_t i, double sv, double sum_t) {
    const double d = bc_delta(sv, sum_t);
    delta_vm[i] = d;
    t_vm[i] = bc_tval(sv, d);
}

__device__ __forceinline__ void msbc_backward_level(const DevGraph &g, int K, const int32_t *srcs,
                                                    const int32_t *depth_vm, const u64 *sigma_vm, double *delta_vm,
                                                    double *t_vm, int level, Tid t) {
    __shared__ int q_v[2][kBlock];
    __shared__ int q_n[2];
    __shared__ double s_w[kBcGroup][kBlock / kWave];
    __shared__ int s_src[kBcGroup];
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    if (tid < kBcGroup) s_src[tid] = tid < K ? srcs[tid] : -1;
    for (int base = t.block * kBlock; base < g.n; base += t.nblocks * kBlock) {
        if (tid < 2) q_n[tid] = 0;
        __syncthreads();
        const int v = base + tid;
        if (v < g.n) {
            unsigned mask = 0;  // sources for which v sits at `level` (and is not the source)
            for (int j = 0; j < K; j++)
                if (depth_vm[(size_t)v * K + j] == level && s_src[j] != v) mask |= 1u << j;
            if (mask) {
                const int beg = g.row_ptr[v], end = g.row_ptr[v + 1];
                const int deg = end - beg;
                if (deg < kBcWaveDeg) {
                    double acc[kBcGroup], sv[kBcGroup];
#pragma unroll
                    for (int j = 0; j < kBcGroup; j++) {
                        acc[j] = 0.0;
                        sv[j] = ((mask >> j) & 1u) ? (double)sigma_vm[(size_t)v * K + j] : 0.0;
                    }
                    for (int e = beg; e < end; e++) {
                        const int w = g.col[e];
#pragma unroll
                        for (int j = 0; j < kBcGroup; j++)
                            if (((mask >> j) & 1u) && depth_vm[(size_t)w * K + j] == level + 1)
                                acc[j] = acc[j] + t_vm[(size_t)w * K + j];
                    }
#pragma unroll
                    for (int j = 0; j < kBcGroup; j++)
                        if ((mask >> j) & 1u) ms_bc_set(delta_vm, t_vm, (size_t)v * K + j, sv[j], acc[j]);
                } else {
                    const int t = deg < kBcBlockDeg ? 0 : 1;
                    q_v[t][atomicAdd(&q_n[t], 1)] = v;
                }
            }
        }
        __syncthreads();
        // one wavefront per vertex
        for (int k = wib; k < q_n[0]; k += kBlock / kWave) {
            const int vv = q_v[0][k];
            unsigned mask = 0;
            for (int j = 0; j < K; j++)
                if (depth_vm[(size_t)vv * K + j] == level && s_src[j] != vv) mask |= 1u << j;
            double acc[kBcGroup], sv[kBcGroup];
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) {
                acc[j] = 0.0;
                sv[j] = ((mask >> j) & 1u) ? (double)sigma_vm[(size_t)vv * K + j] : 0.0;
            }
            for (int e = g.row_ptr[vv] + lane; e < g.row_ptr[vv + 1]; e += kWave) {
                const int w = g.col[e];
#pragma unroll
                for (int j = 0; j < kBcGroup; j++)
                    if (((mask >> j) & 1u) && depth_vm[(size_t)w * K + j] == level + 1)
                        acc[j] = acc[j] + t_vm[(size_t)w * K + j];
            }
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) {
                const double r = wave_sum(acc[j]);
                if (lane == 0 && ((mask >> j) & 1u)) ms_bc_set(delta_vm, t_vm, (size_t)vv * K + j, sv[j], r);
            }
        }
        // the whole workgroup per vertex
        for (int k = 0; k < q_n[1]; k++) {
            const int vv = q_v[1][k];
            unsigned mask = 0;
            for (int j = 0; j < K; j++)
                if (depth_vm[(size_t)vv * K + j] == level && s_src[j] != vv) mask |= 1u << j;
            double acc[kBcGroup], sv[kBcGroup];
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) {
                acc[j] = 0.0;
                sv[j] = ((mask >> j) & 1u) ? (double)sigma_vm[(size_t)vv * K + j] : 0.0;
            }
            for (int e = g.row_ptr[vv] + tid; e < g.row_ptr[vv + 1]; e += kBlock) {
                const int w = g.col[e];
#pragma unroll
                for (int j = 0; j < kBcGroup; j++)
                    if (((mask >> j) & 1u) && depth_vm[(size_t)w * K + j] == level + 1)
                        acc[j] = acc[j] + t_vm[(size_t)w * K + j];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBcGroup; j++) {
                const double r = wave_sum(acc[j]);
                if (lane == 0) s_w[j][wib] = r;
            }
            __syncthreads();
            if (tid < kBcGroup && ((mask >> tid) & 1u)) {
                double t = 0.0;
                for (int w = 0; w < kBlock / kWave; w++) t += s_w[tid][w];
                ms_bc_set(delta_vm, t_vm, (size_t)vv * K + tid, (double)sigma_vm[(size_t)vv * K + tid], t);
            }
        }
        __syncthreads();
    }
}

// ---- one launch per level (unfused schedules) ---------------------------------------------
__global__ __launch_bounds__(kBlock) void k_msbfs_pull(DevGraph g, int K, u64 all, u64 *visited, const u64 *front,
                                                       u64 *next, int32_t *depth_vm, int level, int32_t *any) {
    msbfs_level(g, K, all, visited, front, next, depth_vm, level, any, Tid::here());
}
__global__ __launch_bounds__(kBlock) void k_msbc_pull(DevGraph g, int K, u64 all, u64 *visited, const u64 *front,
                                                      u64 *next, int32_t *depth_vm, u64 *sigma_vm, int level,
                                                      int32_t *flags /* [0] any, [1] overflow */) {
    msbc_level(g, K, all, visited, front, next, depth_vm, sigma_vm, level, flags, flags + 1, Tid::here());
}
__global__ __launch_bounds__(kBlock) void k_msbc_backward(DevGraph g, int K, const int32_t *srcs,
                                                          const int32_t *depth_vm, const u64 *sigma_vm,
                                                          double *delta_vm, double *t_vm, int level) {
    msbc_backward_level(g, K, srcs, depth_vm, sigma_vm, delta_vm, t_vm, level, Tid::here());
}

// ---- one persistent launch per batch (fused schedules): levels separated by grid barriers --
// flags: [0..2] "some vertex found a new source" per level (rotating), [3] path
// count overflow, [4] levels run
struct MsPullArgs {
    DevGraph g;
    int K;
    u64 all;
    u64 *visited, *f0, *f1;
    int32_t *depth_vm;
    u64 *sigma_vm;      // BC only
    double *delta_vm;   // BC only
    double *t_vm;       // BC only: (1 + delta) / sigma
    const int32_t *srcs;
    int32_t *flags;
    GridBarrier bar;
};

template <bool BC>
__global__ __launch_bounds__(kBlock) void k_ms_pull_fused(MsPullArgs a) {
    const Tid t = Tid::here();
    GridBarrier bar = a.bar;
    const bool lead = t.block == 0 && threadIdx.x == 0;
    int level = 1;
    bool ok = true;
    for (;; level++) {
        const u64 *front = (level & 1) ? a.f0 : a.f1;
        u64 *next = (level & 1) ? a.f1 : a.f0;
        int32_t *any = a.flags + level % 3;
        if (lead) __hip_atomic_store(a.flags + (level + 1) % 3, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (BC)
            msbc_level(a.g, a.K, a.all, a.visited, front, next, a.depth_vm, a.sigma_vm, level, any, a.flags + 3, t);
        else
            msbfs_level(a.g, a.K, a.all, a.visited, front, next, a.depth_vm, level, any, t);
        if (!grid_sync(bar)) { ok = false; break; }
        if (load_relaxed(any) == 0) break;
    }
    // levels 0 .. level-1 hold vertices
    if constexpr (BC) {
        for (int L = level - 1; ok && L >= 0; L--) {
            msbc_backward_level(a.g, a.K, a.srcs, a.depth_vm, a.sigma_vm, a.delta_vm, a.t_vm, L, t);
            if (!grid_sync(bar)) ok = false;
        }
    }
    if (lead) a.flags[4] = level;
}

struct MsBuffers {
    u64 *visited, *front, *next;
    int32_t *depth_vm;
};

static MsBuffers ms_buffers(Workspace &ws, int n, int K) {
    ws.aux_u64[0].ensure(n);
    ws.aux_u64[1].ensure(n);
    ws.aux_u64[2].ensure(n);
    ws.aux_i32[3].ensure((size_t)n * (K > 0 ? K : 1));
    return MsBuffers{ws.aux_u64[0].p, ws.aux_u64[1].p, ws.aux_u64[2].p, ws.aux_i32[3].p};
}

// The batch's levels (and, for BC, its backward levels) in one persistent
// launch; returns the number of levels run. Flags land in ws.h_i32[0..7].
template <bool BC>
static int ms_pull_persistent(Ctx &c, Graph &G, Workspace &ws, int K, u64 all, const MsBuffers &b, u64 *sig,
                              double *del, double *tv, const int32_t *srcs) {
    const void *kern = (const void *)k_ms_pull_fused<BC>;
    // every level sweeps all vertices: many waves per compute unit hide the
    // gathers' latency, at a barrier cost that grows with the workgroups
    const int blocks = fused_grid(kern, 4, c.num_cus);
    MsPullArgs a{G.view(), K, all, b.visited, b.front, b.next, b.depth_vm, sig, del, tv, srcs, ws.counters.p,
                 prepare_barrier(c, ws, blocks)};
    void *args[] = {&a};
    launch_cooperative(c, kern, blocks, args);
    check_barrier(c, ws);
    GG_HIP(hipMemcpyAsync(ws.h_i32.p, ws.counters.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    return ws.h_i32.p[4];
}

void msbfs_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &sch, int32_t *depth, hipStream_t stream,
               gg_stats *st) {
    // PUSH without a hybrid switch: the sparse-queue loop (one barrier per
    // level); otherwise the bit-packed PULL sweep below
    if (!sch.hybrid && sch.s1.direction == GG_PUSH) {
        msbfs_push_run(G, srcs, k, depth, stream, st);
        return;
    }
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    if (k == 0) { scope.finish(); return; }
    Lease ws(G);
    const DevGraph g = G.view();
    const int n = g.n;
    MsBuffers b = ms_buffers(*ws, n, k);
    ws->counters.ensure(64);
    ws->h_i32.ensure(16);
    DevBuf<int32_t> dsrc;
    dsrc.ensure(64);
    GG_HIP(hipMemcpyAsync(dsrc.p, srcs, sizeof(int32_t) * k, hipMemcpyHostToDevice, c.s));
    hipLaunchKernelGGL(k_ms_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, n, k, dsrc.p, b.visited,
                       b.front, b.depth_vm, (u64 *)nullptr, (double *)nullptr);
    GG_CHECK_LAUNCH();
    c.launches++;
    const u64 all = k == 64 ? ~0ull : ((1ull << k) - 1);
    if (sch.s1.kernel_fusion) {
        fill_i32(c, ws->counters.p, 8, 0);
        const int levels = ms_pull_persistent<false>(c, G, *ws, k, all, b, nullptr, nullptr, nullptr, nullptr);
        if (st) { st->iterations = levels; st->pull_iterations = levels; st->fused = 1; }
    } else {
        for (int level = 1;; level++) {
            fill_i32(c, ws->counters.p, 1, 0);
            hipLaunchKernelGGL(k_msbfs_pull, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, k, all,
                               b.visited, b.front, b.next, b.depth_vm, level, ws->counters.p);
            GG_CHECK_LAUNCH();
            c.launches++;
            std::swap(b.front, b.next);
            if (st) { st->iterations++; st->pull_iterations++; }
            if (read_i32(c, ws->counters.p, ws->h_i32.p) == 0) break;
        }
    }
    hipLaunchKernelGGL((k_ms_transpose<int32_t, int32_t>), dim3(blocks_for(n, 64, 16384)), dim3(kBlock), 0, c.s,
                       b.depth_vm, n, k, depth, 0);
    GG_CHECK_LAUNCH();
    c.launches++;
    GG_HIP(hipStreamSynchronize(c.s));
    scope.finish();
}

void msbc_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &sch, uint64_t *sigma_out, float *delta_out,
              hipStream_t stream, gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    StatsScope scope(st, c);
    if (k == 0) { scope.finish(); return; }
    Lease ws(G);
    const DevGraph g = G.view();
    const int n = g.n;
    ws->counters.ensure(64);
    ws->h_i32.ensure(16);
    DevBuf<int32_t> dsrc;
    dsrc.ensure(64);
    GG_HIP(hipMemcpyAsync(dsrc.p, srcs, sizeof(int32_t) * k, hipMemcpyHostToDevice, c.s));
    for (int j0 = 0; j0 < k; j0 += kBcGroup) {
        const int K = std::min(kBcGroup, k - j0);
        MsBuffers b = ms_buffers(*ws, n, K);
        ws->aux_u64[0].ensure(n);
        DevBuf<u64> &sig = ws->ms_sigma;
        sig.ensure((size_t)n * K);
        DevBuf<double> &del = ws->aux_f64[1];
        del.ensure((size_t)n * K);
        DevBuf<double> &tv = ws->aux_f64[0];  // (1 + delta) / sigma, written with delta
        tv.ensure((size_t)n * K);
        hipLaunchKernelGGL(k_ms_init, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, n, K, dsrc.p + j0,
                           b.visited, b.front, b.depth_vm, sig.p, del.p);
        GG_CHECK_LAUNCH();
        c.launches++;
        const u64 all = (1ull << K) - 1;
        if (sch.s1.kernel_fusion) {
            fill_i32(c, ws->counters.p, 8, 0);
            const int levels = ms_pull_persistent<true>(c, G, *ws, K, all, b, sig.p, del.p, tv.p, dsrc.p + j0);
            if (st) { st->iterations += levels; st->pull_iterations += levels; st->fused = 1; }
            require(ws->h_i32.p[3] == 0, GG_ERR_OVERFLOW, "a shortest-path count exceeds 2^64-1");
        } else {
            int levels = 1;  // levels present: 0 .. levels-1
            for (int level = 1;; level++) {
                fill_i32(c, ws->counters.p, 2, 0);
                hipLaunchKernelGGL(k_msbc_pull, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, K, all,
                                   b.visited, b.front, b.next, b.depth_vm, sig.p, level, ws->counters.p);
                GG_CHECK_LAUNCH();
                c.launches++;
                std::swap(b.front, b.next);
                if (st) { st->iterations++; st->pull_iterations++; }
                GG_HIP(hipMemcpyAsync(ws->h_i32.p, ws->counters.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
                GG_HIP(hipStreamSynchronize(c.s));
                require(ws->h_i32.p[1] == 0, GG_ERR_OVERFLOW, "a shortest-path count exceeds 2^64-1");
                if (ws->h_i32.p[0] == 0) break;
                levels = level + 1;
            }
            // from the deepest level (no successors: delta 0, t = 1/sigma) up
            for (int level = levels - 1; level >= 0; level--) {
                hipLaunchKernelGGL(k_msbc_backward, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, K,
                                   dsrc.p + j0, b.depth_vm, sig.p, del.p, tv.p, level);
                GG_CHECK_LAUNCH();
                c.launches++;
            }
        }
        hipLaunchKernelGGL((k_ms_transpose<u64, u64>), dim3(blocks_for(n, 64, 16384)), dim3(kBlock), 0, c.s, sig.p, n,
                           K, reinterpret_cast<u64 *>(sigma_out), j0);
        GG_CHECK_LAUNCH();
        hipLaunchKernelGGL((k_ms_transpose<double, float>), dim3(blocks_for(n, 64, 16384)), dim3(kBlock), 0, c.s,
                           del.p, n, K, delta_out, j0);
        GG_CHECK_LAUNCH();
        c.launches += 2;
    }
    GG_HIP(hipStreamSynchronize(c.s));
    scope.finish();
}

}  // namespace gg
