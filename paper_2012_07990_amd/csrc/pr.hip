// PageRank: a topology-driven loop that applies every edge every round
// (Evaluation section, "Algorithms"). Round t computes, for every vertex v,
//   rank'(v) = (1-d)/n + d * ( sum_{u in N(v)} rank(u)/deg(u) + D/n )
// where D is the rank held by zero-degree vertices (spread uniformly; dropped
// with GG_PR_NO_DANGLING). contrib(u) = rank(u)/deg(u) is produced by the
// previous round's vertex apply, together with the next round's D.
//
// Edge traversal forms:
//   PULL VERTEX_BASED  one lane per vertex, neighbours summed in CSR order
//   PULL WM            one wavefront per vertex, lane-strided sums reduced by
//                      a fixed butterfly
//   PULL ETWC          the ETWC stages of a workgroup accumulate per-vertex
//                      sums in LDS (one entry per vertex per stage, stages
//                      separated by barriers, so the order is fixed)
//   PULL STRICT        every workgroup takes the same number of edges; rows
//                      that cross a chunk boundary are completed from the
//                      chunks' head/tail partial sums in the vertex apply.
//                      Each workgroup keeps a copy of the contributions of
//                      the segment's kPrHotK (at most) highest-degree sources in LDS
//                      (refreshed by the vertex apply every round): edges
//                      from those sources read LDS instead of issuing a
//                      random 4-byte global gather (the same values in the
//                      same order, so the sums are unchanged)
//   PUSH EDGE_ONLY     every edge adds contrib(src) to acc(dst) atomically
//   PUSH EDGE_ONLY+EB  the same over the EdgeBlocked COO, one launch per
//                      destination segment (the edge processing algorithm)
// Ranks and contributions are stored in FP32; every neighbour sum is
// accumulated in FP64 (a hub's thousands of terms would otherwise lose
// ~1e-5 absolute). Every PULL form is deterministic; the PUSH forms use FP64
// atomic adds, whose order varies.
#include <algorithm>
#include <cstdio>

#include "algos.hpp"
#include "lb.hpp"

namespace gg {

constexpr int kPrChunk = kWave * 8;   // STRICT: edges per chunk (one wavefront's)
constexpr int kPrWaves = 16;          // STRICT: wavefronts per workgroup
constexpr int kPrHotK = 12288;        // STRICT: highest-degree sources per segment cached in LDS (48 KB)
constexpr int kHotBins = 4096;        // degree histogram bins (the last one collects the rest)

struct PrArgs {
    DevGraph g;
    const float *contrib_in;
    float *contrib_out;
    float *rank_out;        // written on the final round only
    float damping;
    const double *D_in;     // dangling mass of the input round
    double *D_out;
    double *partials;       // per-block dangling partial sums (reduced by k_pr_dangling)
    int dangling;           // 0: drop the dangling mass
    double *acc;            // STRICT / PUSH accumulators (reset after read)
    const int32_t *hot_slot;  // STRICT LDS cache: slot of each cached source (-1: not cached)
    float *hot_out;           // the cached sources' contributions, by slot
};

__device__ __forceinline__ double pr_base(const PrArgs &a) {
    const double n = (double)a.g.n, d = (double)a.damping;
    return (1.0 - d) / n + d * (a.dangling ? *a.D_in : 0.0) / n;
}

__device__ __forceinline__ void pr_apply(const PrArgs &a, int v, double base, double acc, int deg, double &dl) {
    const float nv = (float)(base + (double)a.damping * acc);
    if (a.rank_out) a.rank_out[v] = nv;
    const float cv = deg > 0 ? nv / (float)deg : 0.f;
    a.contrib_out[v] = cv;
    if (a.hot_slot) {
        const int sl = a.hot_slot[v];
        if (sl >= 0) a.hot_out[sl] = cv;
    }
    if (deg == 0) dl += (double)nv;
}

// Block sum of the dangling ranks into the block's partial; k_pr_dangling
// reduces the partials after the kernel (a kernel boundary orders them, with
// no per-workgroup agent-scope fence and ticket).
__device__ void pr_finish(const PrArgs &a, double dl) {
    __shared__ double s_w[kBlock / kWave];
    dl = wave_sum(dl);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = dl;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < kBlock / kWave; w++) t += s_w[w];
        a.partials[blockIdx.x] = t;
    }
}

// D_out = the sum of `count` block partials, in a fixed order
__global__ __launch_bounds__(kBlock) void k_pr_dangling(const double *partials, int count, double *D_out) {
    __shared__ double s_w[kBlock / kWave];
    double t = 0;
    for (int i = threadIdx.x; i < count; i += kBlock) t += partials[i];
    t = wave_sum(t);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int w = 0; w < kBlock / kWave; w++) s += s_w[w];
        *D_out = s;
    }
}

// round 0: rank = 1/n
__global__ __launch_bounds__(kBlock) void k_pr_init(PrArgs a) {
    const float r0 = (float)(1.0 / (double)a.g.n);
    double dl = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < a.g.n; v += gridDim.x * kBlock) {
        const int deg = a.g.row_ptr[v + 1] - a.g.row_ptr[v];
        if (a.rank_out) a.rank_out[v] = r0;
        const float cv = deg > 0 ? r0 / (float)deg : 0.f;
        a.contrib_out[v] = cv;
        if (a.hot_slot) {
            const int sl = a.hot_slot[v];
            if (sl >= 0) a.hot_out[sl] = cv;
        }
        if (deg == 0) dl += (double)r0;
        if (a.acc) a.acc[v] = 0.0;
    }
    pr_finish(a, dl);
}

__global__ __launch_bounds__(kBlock) void k_pr_pull_vp(PrArgs a) {
    const double base = pr_base(a);
    double dl = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < a.g.n; v += gridDim.x * kBlock) {
        const int beg = a.g.in_row_ptr[v], end = a.g.in_row_ptr[v + 1];
        double s = 0.0;
        for (int e = beg; e < end; e++) s += (double)a.contrib_in[a.g.in_col[e]];
        pr_apply(a, v, base, s, a.g.row_ptr[v + 1] - a.g.row_ptr[v], dl);
    }
    pr_finish(a, dl);
}

__global__ __launch_bounds__(kBlock) void k_pr_pull_wm(PrArgs a) {
    const double base = pr_base(a);
    const int lane = lane_id(), wpb = kBlock / kWave;
    double dl = 0;
    for (int v = blockIdx.x * wpb + threadIdx.x / kWave; v < a.g.n; v += gridDim.x * wpb) {
        const int beg = a.g.in_row_ptr[v], end = a.g.in_row_ptr[v + 1];
        double s = 0.0;
        for (int e = beg + lane; e < end; e += kWave) s += (double)a.contrib_in[a.g.in_col[e]];
        s = wave_sum(s);
        if (lane == 0) pr_apply(a, v, base, s, a.g.row_ptr[v + 1] - a.g.row_ptr[v], dl);
    }
    pr_finish(a, dl);
}

__device__ __forceinline__ double block_sum_d(double x, double *s_tmp) {
    x = wave_sum(x);
    __syncthreads();
    if (lane_id() == 0) s_tmp[threadIdx.x / kWave] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) t += s_tmp[w];
    return t;
}

__global__ __launch_bounds__(kBlock) void k_pr_pull_etwc(PrArgs a) {
    __shared__ int q_beg[3][kBlock], q_end[3][kBlock], q_slot[3][kBlock];
    __shared__ int q_n[3];
    __shared__ double s_acc[kBlock];
    __shared__ double s_tmp[kBlock / kWave];
    const double base = pr_base(a);
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    double dl = 0;
    for (int vb = blockIdx.x * kBlock; vb < a.g.n; vb += gridDim.x * kBlock) {
        if (tid < 3) q_n[tid] = 0;
        s_acc[tid] = 0.0;
        __syncthreads();
        const int v = vb + tid;
        int deg = 0;  // out-degree (the contribution's divisor); the sums run over in-edges
        if (v < a.g.n) {
            int beg = a.g.in_row_ptr[v];
            const int end = a.g.in_row_ptr[v + 1];
            deg = a.g.row_ptr[v + 1] - a.g.row_ptr[v];
            int size = end - beg;
            const int s2 = (size / kBlock) * kBlock;
            if (s2 > 0) {
                const int k = atomicAdd(&q_n[2], 1);
                q_beg[2][k] = beg; q_end[2][k] = beg + s2; q_slot[2][k] = tid;
                beg += s2; size -= s2;
            }
            const int s1 = (size / kWave) * kWave;
            if (s1 > 0) {
                const int k = atomicAdd(&q_n[1], 1);
                q_beg[1][k] = beg; q_end[1][k] = beg + s1; q_slot[1][k] = tid;
                beg += s1; size -= s1;
            }
            if (size > 0) {
                const int k = atomicAdd(&q_n[0], 1);
                q_beg[0][k] = beg; q_end[0][k] = end; q_slot[0][k] = tid;
            }
        }
        __syncthreads();
        // stage 0: one lane per entry (sequential CSR order)
        for (int k = tid; k < q_n[0]; k += kBlock) {
            double s = 0.0;
            for (int e = q_beg[0][k]; e < q_end[0][k]; e++) s += (double)a.contrib_in[a.g.in_col[e]];
            s_acc[q_slot[0][k]] += s;
        }
        __syncthreads();
        // stage 1: one wavefront per entry
        for (int k = wib; k < q_n[1]; k += kBlock / kWave) {
            double s = 0.0;
            for (int e = q_beg[1][k] + lane; e < q_end[1][k]; e += kWave) s += (double)a.contrib_in[a.g.in_col[e]];
            s = wave_sum(s);
            if (lane == 0) s_acc[q_slot[1][k]] += s;
        }
        __syncthreads();
        // stage 2: the whole workgroup per entry
        for (int k = 0; k < q_n[2]; k++) {
            double s = 0.0;
            for (int e = q_beg[2][k] + tid; e < q_end[2][k]; e += kBlock) s += (double)a.contrib_in[a.g.in_col[e]];
            s = block_sum_d(s, s_tmp);
            if (tid == 0) s_acc[q_slot[2][k]] += s;
        }
        __syncthreads();
        if (v < a.g.n) pr_apply(a, v, base, s_acc[tid], deg, dl);
        __syncthreads();
    }
    pr_finish(a, dl);
}

// owner row of edge e: the last r with row_ptr[r] <= e
__device__ __forceinline__ int owner_row(const int32_t *rp, int n, long long e) {
    int lo = 0, hi = n;  // rp[lo] <= e < rp[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// once per graph: rows[2c] = owner of chunk c's first edge, rows[2c+1] = owner
// of its last edge
__global__ __launch_bounds__(kBlock) void k_pr_partition(const int32_t *rp, int n, long long m, long long nchunks,
                                                         int32_t *rows) {
    for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (long long)gridDim.x * kBlock) {
        const long long E0 = c * kPrChunk, E1 = (E0 + kPrChunk < m) ? E0 + kPrChunk : m;
        rows[2 * c] = owner_row(rp, n, E0);
        rows[2 * c + 1] = owner_row(rp, n, E1 - 1);
    }
}

// LDS writes of one wavefront made visible to its other lanes (no workgroup
// barrier: the wavefronts of a workgroup run their chunks independently)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// STRICT: chunk c holds edges [c*C, c*C + C) of a (segment) CSR and belongs to
// one wavefront. Rows entirely inside a chunk add their sum to accum; the
// chunk's first and last rows also leave their in-chunk partial sums in
// head[c] / tail[c], which k_pr_fixup adds for the rows that span chunks.
// With HK > 0 the column entries of cached sources hold ~slot and their values
// come from an LDS copy of the segment's nhot (<= HK, a multiple of 4) entries
// of `hot`, loaded once per workgroup (the grid is sized to stay resident).
template <int HK>
__global__ __launch_bounds__(kWave *kPrWaves) __attribute__((amdgpu_waves_per_eu(8))) void k_pr_strict_chunks(
    const int32_t *rp, const int32_t *col, long long m, const float *contrib, const float *hot, int nhot,
    const int32_t *chunk_rows, double *accum, double *head, double *tail, long long nchunks) {
    __shared__ float vals[kPrWaves][kPrChunk];
    __shared__ float4 hot_s4[HK > 0 ? HK / 4 : 1];
    const float *hot_s = reinterpret_cast<const float *>(hot_s4);
    const int lane = lane_id(), wib = (int)threadIdx.x / kWave;
    if constexpr (HK > 0) {
        const float4 *h4 = reinterpret_cast<const float4 *>(hot);
        for (int i = threadIdx.x; i < nhot / 4; i += kWave * kPrWaves) hot_s4[i] = h4[i];
        __syncthreads();
    }
    float *cv = vals[wib];
    // Column loads, then gathers, without branches in between (a conditional
    // per edge made the compiler wait for each load in turn); edges past a
    // chunk's end re-read its last edge and are not stored. The column stream
    // is read once: non-temporal loads keep it from evicting the segment's
    // contributions from L2. The loop is software-pipelined: the next
    // chunk's columns are requested as soon as this chunk's gathers are, so
    // they arrive during this chunk's reduction.
    constexpr int kPer = kPrChunk / kWave;
    const long long cstride = (long long)gridDim.x * kPrWaves;
    long long c = (long long)blockIdx.x * kPrWaves + wib;
    int cnext[kPer];
    auto load_cols = [&](long long cc) {
        const long long F0 = cc * kPrChunk, F1 = (F0 + kPrChunk < m) ? F0 + kPrChunk : m;
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const long long e = F0 + k * kWave + lane;
            cnext[k] = __builtin_nontemporal_load(&col[e < F1 ? e : F1 - 1]);
        }
    };
    if (c < nchunks) load_cols(c);
    for (; c < nchunks; c += cstride) {
        const long long E0 = c * kPrChunk, E1 = (E0 + kPrChunk < m) ? E0 + kPrChunk : m;
        const int r0 = chunk_rows[2 * c], r1 = chunk_rows[2 * c + 1];
        int cidx[kPer];
        float cval[kPer];
#pragma unroll
        for (int k = 0; k < kPer; k++) cidx[k] = cnext[k];
        // the offsets of the chunk's first 128 rows travel with its gathers
        // (a row past r1 re-reads r1's): vector loads complete in order, so a
        // row offset requested after the next chunk's columns would make the
        // reduction wait for those too
        const int rf = r0 + lane <= r1 ? r0 + lane : r1;
        const int rs = r0 + kWave + lane <= r1 ? r0 + kWave + lane : r1;
        const int rb_first = rp[rf], re_first = rp[rf + 1];
        const int rb_second = rp[rs], re_second = rp[rs + 1];
        if constexpr (HK > 0) {
            // a cached source's lane reads contrib[0] (one shared line for the
            // wavefront) and takes the LDS value; the rest read LDS entry 0
            float gv[kPer];
#pragma unroll
            for (int k = 0; k < kPer; k++) gv[k] = contrib[cidx[k] >= 0 ? cidx[k] : 0];
#pragma unroll
            for (int k = 0; k < kPer; k++) {
                const int i = cidx[k];
                const float hv = hot_s[i >= 0 ? 0 : ~i];
                cval[k] = i >= 0 ? gv[k] : hv;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPer; k++) cval[k] = contrib[cidx[k]];
        }
        if (c + cstride < nchunks) load_cols(c + cstride);
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const long long e = E0 + k * kWave + lane;
            if (e < E1) cv[e - E0] = cval[k];
        }
        wave_lds_sync();
        // short rows (< 32 in-chunk edges): one lane each, in CSR order; long
        // rows: the whole wavefront, lane-strided sums reduced by a butterfly.
        // A row inside the chunk adds its sum to accum with an atomic whose
        // result is not awaited: within one launch (one source segment) no
        // other add reaches that row, so the value equals a read-modify-write
        // in launch order, without the wait for the read
        for (int rbase = r0; rbase <= r1; rbase += kWave) {
            const int r = rbase + lane;
            int lo = 0, hi = 0, whole = 0;
            if (r <= r1) {
                const long long rb = rbase == r0 ? rb_first : rbase == r0 + kWave ? rb_second : rp[r];
                const long long re = rbase == r0 ? re_first : rbase == r0 + kWave ? re_second : rp[r + 1];
                lo = (int)((rb > E0 ? rb : E0) - E0);
                hi = (int)((re < E1 ? re : E1) - E0);
                whole = rb >= E0 && re <= E1;
            }
            const bool lng = hi - lo >= 32;
            if (r <= r1 && !lng) {
                // four LDS reads in flight per step, added in row order (the
                // additions, and so the rounding, are the plain loop's)
                double sum = 0.0;
                int i = lo;
                for (; i + 4 <= hi; i += 4) {
                    const float x0 = cv[i], x1 = cv[i + 1], x2 = cv[i + 2], x3 = cv[i + 3];
                    sum += (double)x0;
                    sum += (double)x1;
                    sum += (double)x2;
                    sum += (double)x3;
                }
                for (; i < hi; i++) sum += (double)cv[i];
                if (whole && hi > lo) (void)atomic_add_f64(&accum[r], sum);
                if (r == r0) head[c] = sum;
                if (r == r1) tail[c] = sum;
            }
            uint64_t lm = __ballot(lng);
            while (lm) {
                const int o = first_lane(lm);
                lm &= lm - 1;
                const int rr = rbase + o, llo = __shfl(lo, o, kWave), lhi = __shfl(hi, o, kWave);
                const int wh = __shfl(whole, o, kWave);
                double sum = 0.0;
                for (int i = llo + lane; i < lhi; i += kWave) sum += (double)cv[i];
                sum = wave_sum(sum);
                if (lane == 0) {
                    if (wh) (void)atomic_add_f64(&accum[rr], sum);
                    if (rr == r0) head[c] = sum;
                    if (rr == r1) tail[c] = sum;
                }
            }
        }
        wave_lds_sync();  // this chunk's reads of cv come before the next chunk's writes
    }
}

// Rows that span chunks: a row that starts inside chunk c and ends beyond it
// is chunk c's last row; its sum is tail[c] + the heads of the chunks it
// covers, in chunk order.
__global__ __launch_bounds__(kBlock) void k_pr_fixup(const int32_t *rp, long long m, const int32_t *chunk_rows,
                                                     const double *head, const double *tail, double *accum,
                                                     long long nchunks) {
    for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (long long)gridDim.x * kBlock) {
        const long long E0 = c * kPrChunk, E1 = (c + 1) * kPrChunk < m ? (c + 1) * kPrChunk : m;
        const int r = chunk_rows[2 * c + 1];
        const long long rb = rp[r], re = rp[r + 1];
        if (re <= E1 || rb < E0) continue;  // fixed up by the chunk where the row starts
        const long long c1 = (re - 1) / kPrChunk;
        // a hub's row covers many chunks: eight head loads are issued ahead of
        // their additions, which keep the chunk order
        double sum = tail[c];
        long long k = c + 1;
        for (; k + 8 <= c1; k += 8) {
            double h[8];
#pragma unroll
            for (int b = 0; b < 8; b++) h[b] = head[k + b];
#pragma unroll
            for (int b = 0; b < 8; b++) sum += h[b];
        }
        for (; k < c1; k++) sum += head[k];
        sum += head[c1];
        accum[r] += sum;
    }
}

// Vertex apply after STRICT chunks or PUSH accumulation: reads the neighbour
// sum from acc and resets it for the next round.
__global__ __launch_bounds__(kBlock) void k_pr_apply(PrArgs a) {
    const double base = pr_base(a);
    double dl = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < a.g.n; v += gridDim.x * kBlock) {
        const int deg = a.g.row_ptr[v + 1] - a.g.row_ptr[v];
        const double s = a.acc[v];
        a.acc[v] = 0.0;
        pr_apply(a, v, base, s, deg, dl);
    }
    pr_finish(a, dl);
}

// ---- PULL EdgeBlocking layout: segment s holds, for every destination row,
// its sources in [s*N, (s+1)*N) (a contiguous piece of the sorted row).
__device__ __forceinline__ int row_lower_bound(const int32_t *col, int lo, int hi, long long x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_seg_count(DevGraph g, int N, int S, int32_t *rp_s) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < g.n; v += gridDim.x * kBlock) {
        const int beg = g.in_row_ptr[v], end = g.in_row_ptr[v + 1];
        int lo = beg;
        for (int s = 0; s < S; s++) {
            const int hi = s == S - 1 ? end : row_lower_bound(g.in_col, lo, end, (long long)(s + 1) * N);
            rp_s[(long long)s * (g.n + 1) + v] = hi - lo;
            lo = hi;
        }
    }
}

// Copy each row's piece in segment s; pieces of 64 or more entries are copied
// by a whole wavefront (a hub's piece would otherwise be one lane's loop).
__global__ __launch_bounds__(kBlock) void k_seg_fill(DevGraph g, int N, int s, const int32_t *rp_s, int32_t *col_s) {
    __shared__ int q_lo[kBlock], q_len[kBlock], q_dst[kBlock];
    __shared__ int nq;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    for (int base = blockIdx.x * kBlock; base < g.n; base += gridDim.x * kBlock) {
        if (tid == 0) nq = 0;
        __syncthreads();
        const int v = base + tid;
        if (v < g.n) {
            const int beg = g.in_row_ptr[v], end = g.in_row_ptr[v + 1];
            const int lo = row_lower_bound(g.in_col, beg, end, (long long)s * N);
            const int hi = row_lower_bound(g.in_col, lo, end, (long long)(s + 1) * N);
            if (hi - lo < kWave) {
                int32_t *dst = col_s + rp_s[v];
                for (int e = lo; e < hi; e++) dst[e - lo] = g.in_col[e];
            } else {
                const int k = atomicAdd(&nq, 1);
                q_lo[k] = lo;
                q_len[k] = hi - lo;
                q_dst[k] = rp_s[v];
            }
        }
        __syncthreads();
        for (int k = wib; k < nq; k += kBlock / kWave)
            for (int i = lane; i < q_len[k]; i += kWave) col_s[q_dst[k] + i] = g.in_col[q_lo[k] + i];
        __syncthreads();
    }
}

// PUSH EDGE_ONLY: acc[dst] += contrib[src] for every CSR entry
__global__ __launch_bounds__(kBlock) void k_pr_push_edges(const int32_t *src, const int32_t *dst, long long lo,
                                                          long long hi, const float *contrib, double *acc) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long e = lo + (long long)blockIdx.x * kBlock + threadIdx.x; e < hi; e += stride)
        atomic_add_f64(&acc[dst[e]], (double)contrib[src[e]]);
}

// ---- STRICT LDS cache of the highest-degree sources of each segment. On a
// symmetric graph a source appears in as many pull rows as its degree, so the
// kPrHotK highest-degree vertices of a segment cover the most gathers.
constexpr int kHotSpan = 8192;  // vertices per workgroup in the histogram pass

// per segment: hist[s][min(deg, kHotBins-1)] += 1 (small bins of the
// workgroup's first segment counted in LDS first)
__global__ __launch_bounds__(kBlock) void k_hot_hist(DevGraph g, int N, int32_t *hist) {
    __shared__ int sh[kBlock];
    const int tid = threadIdx.x;
    const long long v0 = (long long)blockIdx.x * kHotSpan;
    const long long v1 = v0 + kHotSpan < g.n ? v0 + kHotSpan : g.n;
    const int s0 = (int)(v0 / N);
    sh[tid] = 0;
    __syncthreads();
    for (long long v = v0 + tid; v < v1; v += kBlock) {
        const int d = g.row_ptr[v + 1] - g.row_ptr[v];
        const int b = d < kHotBins - 1 ? d : kHotBins - 1;
        const int sg = (int)(v / N);
        if (sg == s0 && b < kBlock) atomicAdd(&sh[b], 1);
        else atomicAdd(&hist[(long long)sg * kHotBins + b], 1);
    }
    __syncthreads();
    if (sh[tid]) atomicAdd(&hist[(long long)s0 * kHotBins + tid], sh[tid]);
}

// per segment: thr[s] = the smallest degree bin t >= 1 such that at most K
// vertices have a bin >= t (the last bin alone may exceed K; slots then run
// out and the rest stay uncached)
__global__ __launch_bounds__(kBlock) void k_hot_threshold(const int32_t *hist, int K, int32_t *thr) {
    constexpr int kPer = kHotBins / kBlock;
    __shared__ int part[kBlock];
    const int32_t *h = hist + (long long)blockIdx.x * kHotBins;
    int t = 0;
    for (int i = 0; i < kPer; i++) t += h[threadIdx.x * kPer + i];
    part[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        int th = 1;
        for (int i = kBlock - 1; i >= 0 && th == 1; i--) {
            if (acc + part[i] <= K) { acc += part[i]; continue; }
            for (int b = i * kPer + kPer - 1; b >= i * kPer; b--) {
                if (acc + h[b] > K) { th = b + 1 < kHotBins ? b + 1 : kHotBins - 1; break; }
                acc += h[b];
            }
        }
        thr[blockIdx.x] = th;
    }
}

// pass 0: every vertex of bin >= thr gets a slot (while the segment has
// slots), the others -1; pass 1: vertices of bin thr-1 fill the slots left
__global__ __launch_bounds__(kBlock) void k_hot_assign(DevGraph g, int N, int K, const int32_t *thr, int pass,
                                                       int32_t *nslot, int32_t *hot_slot) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < g.n; v += gridDim.x * kBlock) {
        const int d = g.row_ptr[v + 1] - g.row_ptr[v];
        const int b = d < kHotBins - 1 ? d : kHotBins - 1;
        const int sg = v / N, t = thr[sg];
        bool want;
        if (pass == 0) {
            want = b >= t;
            if (!want) hot_slot[v] = -1;
        } else {
            want = t > 1 && b == t - 1;
        }
        if (!want) continue;
        const int k = atomicAdd(&nslot[sg], 1);
        if (k < K) hot_slot[v] = sg * K + k;
        else if (pass == 0) hot_slot[v] = -1;
    }
}

// the pull columns with every cached source u replaced by ~(its slot within
// u's segment)
__global__ __launch_bounds__(kBlock) void k_hot_encode(const int32_t *col, long long m, int N, int K,
                                                       const int32_t *hot_slot, int32_t *hcol) {
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < m; e += (long long)gridDim.x * kBlock) {
        const int u = col[e];
        const int sl = hot_slot[u];
        hcol[e] = sl >= 0 ? ~(sl - (u / N) * K) : u;
    }
}

static void build_hot_cache(Ctx &c, const DevGraph &g, PullBlocked &pb) {
    const int n = g.n, S = pb.S, N = pb.S == 1 ? std::max(n, 1) : pb.N;
    // slots per segment: no more than the segment has vertices (rounded up to
    // whole float4 loads), so narrow segments keep the tables O(n)
    const int K = (int)std::min<long long>(kPrHotK, ((long long)N + 3) / 4 * 4);
    DevBuf<int32_t> hist, thr, nslot;
    hist.ensure((size_t)S * kHotBins);
    thr.ensure(S);
    nslot.ensure(S);
    fill_i32(c, hist.p, (long long)S * kHotBins, 0);
    fill_i32(c, nslot.p, S, 0);
    pb.hot_slot.ensure(std::max(n, 1));
    pb.hcol.ensure((size_t)std::max<long long>(g.m, 1));
    hipLaunchKernelGGL(k_hot_hist, dim3(blocks_for(n, kHotSpan)), dim3(kBlock), 0, c.s, g, N, hist.p);
    GG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_hot_threshold, dim3(S), dim3(kBlock), 0, c.s, hist.p, K, thr.p);
    GG_CHECK_LAUNCH();
    for (int pass = 0; pass < 2; pass++) {
        hipLaunchKernelGGL(k_hot_assign, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, N, K,
                           thr.p, pass, nslot.p, pb.hot_slot.p);
        GG_CHECK_LAUNCH();
    }
    if (g.m > 0) {
        hipLaunchKernelGGL(k_hot_encode, dim3(blocks_for(g.m, kBlock, 16384)), dim3(kBlock), 0, c.s, pb.col_ptr,
                           (long long)g.m, N, K, pb.hot_slot.p, pb.hcol.p);
        GG_CHECK_LAUNCH();
    }
    GG_HIP(hipStreamSynchronize(c.s));  // the temporaries are freed on return
    pb.hot_k = K;
}

// Build (once per graph and segment width) the STRICT pull layout: S = 1 uses
// the graph's own CSR; S > 1 the source-segmented CSRs.
static PullBlocked &pull_layout(Ctx &c, Graph &G, int N) {
    const DevGraph g = G.view();
    const int n = g.n;
    const int S = (int)std::max<long long>(1, ((long long)n + N - 1) / N);
    const int key = S == 1 ? 0 : N;
    std::lock_guard<std::mutex> lk(G.mu);
    auto it = G.pull_eb.find(key);
    if (it != G.pull_eb.end()) return *it->second;
    auto pb = std::make_unique<PullBlocked>();
    pb->N = N;
    pb->S = S;
    if (S == 1) {
        pb->rp_ptr = g.in_row_ptr;
        pb->col_ptr = g.in_col;
        pb->m_s = {(long long)g.m};
        pb->col_base = {0};
    } else {
        pb->rp.ensure((size_t)S * (n + 1));
        pb->col.ensure((size_t)std::max<long long>(g.m, 1));
        hipLaunchKernelGGL(k_seg_count, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, N, S, pb->rp.p);
        GG_CHECK_LAUNCH();
        DevBuf<long long> part;
        part.ensure(exclusive_scan_partials(n));
        std::vector<int32_t> tot(S);
        for (int s = 0; s < S; s++) {
            exclusive_scan_i32(c, pb->rp.p + (size_t)s * (n + 1), n, part.p);
            GG_HIP(hipMemcpyAsync(&tot[s], pb->rp.p + (size_t)s * (n + 1) + n, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  c.s));
        }
        GG_HIP(hipStreamSynchronize(c.s));
        long long base = 0;
        for (int s = 0; s < S; s++) {
            pb->m_s.push_back(tot[s]);
            pb->col_base.push_back(base);
            hipLaunchKernelGGL(k_seg_fill, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, g, N, s,
                               pb->rp.p + (size_t)s * (n + 1), pb->col.p + base);
            GG_CHECK_LAUNCH();
            base += tot[s];
        }
        pb->rp_ptr = pb->rp.p;
        pb->col_ptr = pb->col.p;
    }
    long long total_chunks = 0;
    for (int s = 0; s < S; s++) {
        pb->chunk_base.push_back(total_chunks);
        const long long nc = (pb->m_s[s] + kPrChunk - 1) / kPrChunk;
        pb->nchunks.push_back(nc);
        total_chunks += nc;
    }
    pb->chunk_rows.ensure((size_t)std::max(2 * total_chunks, 2ll));
    build_hot_cache(c, g, *pb);
    for (int s = 0; s < S; s++) {
        if (pb->nchunks[s] == 0) continue;
        hipLaunchKernelGGL(k_pr_partition, dim3(blocks_for(pb->nchunks[s], kBlock, 4096)), dim3(kBlock), 0, c.s,
                           pb->rp_ptr + (S == 1 ? 0 : (size_t)s * (n + 1)), n, pb->m_s[s], pb->nchunks[s],
                           pb->chunk_rows.p + 2 * pb->chunk_base[s]);
        GG_CHECK_LAUNCH();
    }
    GG_HIP(hipStreamSynchronize(c.s));
    auto &ref = *pb;
    G.pull_eb[key] = std::move(pb);
    return ref;
}

void ensure_coo(Ctx &c, Graph &G);

double pull_layout_prepare(Graph &G, int32_t seg_vertices, hipStream_t stream) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    const int N = seg_vertices;
    const int S = (int)std::max<long long>(1, ((long long)G.n + N - 1) / N);
    {
        std::lock_guard<std::mutex> lk(G.mu);
        if (G.pull_eb.count(S == 1 ? 0 : N)) return 0.0;
    }
    ensure_transpose(c, G);
    hipEvent_t e0, e1;
    GG_HIP(hipEventCreate(&e0));
    GG_HIP(hipEventCreate(&e1));
    GG_HIP(hipEventRecord(e0, c.s));
    pull_layout(c, G, N);
    GG_HIP(hipEventRecord(e1, c.s));
    GG_HIP(hipEventSynchronize(e1));
    float ms = 0;
    GG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

// resident workgroups of a STRICT kernel (each loads its LDS copy once)
template <int HK>
static long long strict_grid(int num_cus) {
    static const int occ = [] {
        int o = 0;
        GG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void *)k_pr_strict_chunks<HK>,
                                                            kWave * kPrWaves, 0));
        return o > 0 ? o : 1;
    }();
    return (long long)occ * num_cus;
}

void pr_run(Graph &G, const gg_schedule &sch, float damping, int iters, uint32_t flags, float *rank,
            hipStream_t stream, gg_stats *st) {
    Ctx c;
    c.s = stream;
    c.num_cus = G.num_cus;
    const gg_simple_schedule &s = sch.s1;
    const bool push = s.direction == GG_PUSH;
    if (push) ensure_coo(c, G);
    else ensure_transpose(c, G);  // directed graphs: the sums run over in-edges
    EdgeBlocked *eb = nullptr;
    if (push && s.edge_blocking) {
        edgeblock_prepare(c, G, s.blocking_size);
        std::lock_guard<std::mutex> lk(G.mu);
        eb = G.eb.at(s.blocking_size).get();
    }
    hipEvent_t e0, e1;
    GG_HIP(hipEventCreate(&e0));
    GG_HIP(hipEventCreate(&e1));
    Lease ws(G);
    const DevGraph g = G.view();
    const int n = g.n;
    const int lb = s.load_balance;
    const unsigned nblk = blocks_for(n, kBlock, (unsigned)G.num_cus * 8);
    const unsigned nblk_wm = blocks_for(n, kBlock / kWave, (unsigned)G.num_cus * 16);
    const unsigned apply_blocks = std::max(nblk, nblk_wm);
    ws->pr_contrib[0].ensure(n);
    ws->pr_contrib[1].ensure(n);
    ws->pr_partial.ensure(apply_blocks + 1);
    ws->pr_dangling.ensure(2);
    const bool strict = !push && lb == GG_LB_STRICT;
    PullBlocked *pb = nullptr;
    if (strict || push) ws->pr_acc.ensure(n);
    if (strict) {
        pb = &pull_layout(c, G, s.edge_blocking ? s.blocking_size : std::max(n, 1));
        long long maxc = 1;
        for (long long x : pb->nchunks) maxc = std::max(maxc, x);
        ws->pr_head.ensure((size_t)maxc);
        ws->pr_tail.ensure((size_t)maxc);
    }
    const bool cached = strict && !(flags & GG_PR_NO_LDS_CACHE) && pb->hot_k > 0;
    if (cached) {
        if (pb->hot_k > kPrHotK || pb->hot_k % 4 != 0)
            throw Error(GG_ERR_DEVICE, "PageRank LDS cache: bad slot count per segment");
        ws->pr_hot[0].ensure((size_t)pb->S * pb->hot_k);
        ws->pr_hot[1].ensure((size_t)pb->S * pb->hot_k);
    }
    KernelTimer kt;
    kt.on = st && (st->flags & GG_STATS_TIME_KERNELS);
    kt.s = c.s;
    const char *kname = push     ? "k_pr_push_edges"
                        : cached ? "k_pr_strict_chunks (LDS cache)"
                        : strict ? "k_pr_strict_chunks"
                        : lb == GG_LB_WM ? "k_pr_pull_wm"
                        : lb == GG_LB_ETWC ? "k_pr_pull_etwc" : "k_pr_pull_vp";
    GG_HIP(hipEventRecord(e0, c.s));

    PrArgs a{};
    a.g = g;
    a.damping = damping;
    a.dangling = (flags & GG_PR_NO_DANGLING) ? 0 : 1;
    a.partials = ws->pr_partial.p;
    a.acc = (strict || push) ? ws->pr_acc.p : nullptr;
    a.hot_slot = cached ? pb->hot_slot.p : nullptr;
    // round 0
    a.contrib_out = ws->pr_contrib[0].p;
    a.hot_out = cached ? ws->pr_hot[0].p : nullptr;
    a.rank_out = iters == 0 ? rank : nullptr;
    a.D_out = ws->pr_dangling.p + 0;
    hipLaunchKernelGGL(k_pr_init, dim3(nblk), dim3(kBlock), 0, c.s, a);
    GG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pr_dangling, dim3(1), dim3(kBlock), 0, c.s, a.partials, (int)nblk, a.D_out);
    GG_CHECK_LAUNCH();
    c.launches += 2;
    for (int t = 0; t < iters; t++) {
        a.contrib_in = ws->pr_contrib[t & 1].p;
        a.contrib_out = ws->pr_contrib[(t + 1) & 1].p;
        a.D_in = ws->pr_dangling.p + (t & 1);
        a.D_out = ws->pr_dangling.p + ((t + 1) & 1);
        a.rank_out = t == iters - 1 ? rank : nullptr;
        const float *hot_in = cached ? ws->pr_hot[t & 1].p : nullptr;
        a.hot_out = cached ? ws->pr_hot[(t + 1) & 1].p : nullptr;
        if (push) {
            if (eb) {
                for (size_t sg = 0; sg + 1 < eb->seg_start.size(); sg++) {
                    const long long lo = eb->seg_start[sg], hi = eb->seg_start[sg + 1];
                    if (hi <= lo) continue;
                    kt.begin();
                    hipLaunchKernelGGL(k_pr_push_edges, dim3(blocks_for(hi - lo, kBlock, 16384)), dim3(kBlock), 0,
                                       c.s, eb->src.p, eb->dst.p, lo, hi, a.contrib_in, a.acc);
                    kt.end();
                    GG_CHECK_LAUNCH();
                    c.launches++;
                }
            } else if (g.m > 0) {
                kt.begin();
                hipLaunchKernelGGL(k_pr_push_edges, dim3(blocks_for(g.m, kBlock, 16384)), dim3(kBlock), 0, c.s,
                                   g.coo_src, g.col, 0ll, (long long)g.m, a.contrib_in, a.acc);
                kt.end();
                GG_CHECK_LAUNCH();
                c.launches++;
            }
            hipLaunchKernelGGL(k_pr_apply, dim3(nblk), dim3(kBlock), 0, c.s, a);
        } else if (strict) {
            for (int sg = 0; sg < pb->S; sg++) {
                const long long nc = pb->nchunks[sg];
                if (nc == 0) continue;
                const int32_t *rp = pb->rp_ptr + (pb->S == 1 ? 0 : (size_t)sg * (n + 1));
                const int32_t *cr = pb->chunk_rows.p + 2 * pb->chunk_base[sg];
                kt.begin();
                const long long groups = (nc + kPrWaves - 1) / kPrWaves;
                if (cached) {
                    hipLaunchKernelGGL((k_pr_strict_chunks<kPrHotK>),
                                       dim3((unsigned)std::min<long long>(groups, strict_grid<kPrHotK>(c.num_cus))),
                                       dim3(kWave * kPrWaves), 0, c.s, rp, pb->hcol.p + pb->col_base[sg],
                                       pb->m_s[sg], a.contrib_in, hot_in + (size_t)sg * pb->hot_k, pb->hot_k, cr,
                                       ws->pr_acc.p, ws->pr_head.p, ws->pr_tail.p, nc);
                } else {
                    hipLaunchKernelGGL((k_pr_strict_chunks<0>),
                                       dim3((unsigned)std::min<long long>(groups, strict_grid<0>(c.num_cus))),
                                       dim3(kWave * kPrWaves), 0, c.s, rp, pb->col_ptr + pb->col_base[sg],
                                       pb->m_s[sg], a.contrib_in, nullptr, 0, cr, ws->pr_acc.p, ws->pr_head.p,
                                       ws->pr_tail.p, nc);
                }
                kt.end();
                GG_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_pr_fixup, dim3(blocks_for(nc, kBlock, 4096)), dim3(kBlock), 0, c.s, rp,
                                   pb->m_s[sg], cr, ws->pr_head.p, ws->pr_tail.p, ws->pr_acc.p, nc);
                GG_CHECK_LAUNCH();
                c.launches += 2;
            }
            hipLaunchKernelGGL(k_pr_apply, dim3(nblk), dim3(kBlock), 0, c.s, a);
        } else if (lb == GG_LB_WM) {
            kt.begin();
            hipLaunchKernelGGL(k_pr_pull_wm, dim3(nblk_wm), dim3(kBlock), 0, c.s, a);
            kt.end();
        } else if (lb == GG_LB_ETWC) {
            kt.begin();
            hipLaunchKernelGGL(k_pr_pull_etwc, dim3(nblk), dim3(kBlock), 0, c.s, a);
            kt.end();
        } else {
            kt.begin();
            hipLaunchKernelGGL(k_pr_pull_vp, dim3(nblk), dim3(kBlock), 0, c.s, a);
            kt.end();
        }
        GG_CHECK_LAUNCH();
        const unsigned nparts = (!push && !strict && lb == GG_LB_WM) ? nblk_wm : nblk;
        hipLaunchKernelGGL(k_pr_dangling, dim3(1), dim3(kBlock), 0, c.s, a.partials, (int)nparts, a.D_out);
        GG_CHECK_LAUNCH();
        c.launches += 2;
    }
    GG_HIP(hipEventRecord(e1, c.s));
    GG_HIP(hipEventSynchronize(e1));
    if (st) {
        const uint32_t fl = st->flags;
        *st = gg_stats{};
        st->flags = fl;
        float ms = 0;
        GG_HIP(hipEventElapsedTime(&ms, e0, e1));
        st->device_ms = ms;
        st->iterations = iters;
        st->launches = c.launches;
        if (fl & GG_STATS_COUNT_EDGES) {
            st->edges_examined = (int64_t)g.m * iters;
            st->vertices_processed = (int64_t)n * iters;
        }
        if (push) st->push_iterations = iters; else st->pull_iterations = iters;
        if (kt.on) {
            st->kernel_launches = (int32_t)kt.ev.size();
            st->kernel_ms = kt.total();
            snprintf(st->kernel_name, sizeof(st->kernel_name), "%s", kname);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace gg
