// Kernel fusion across iterations (GPU Optimization Space section, "Kernel
// Fusion across Iterations"; GPU Backend Implementation section): the whole
// while-loop runs inside one persistent launch whose workgroups are all
// co-resident, the operators run as grid-stride __device__ calls, and the
// iterations are separated by a grid-wide barrier. Loop state lives in
// device memory.
//
// The barrier is agent-scope: each XCD of the chip has its own L2, so the
// arrival is a release (dirty lines written back) and the departure an
// acquire (stale lines dropped) at agent scope. Every wait is bounded: if a
// workgroup spins for longer than the limit the barrier raises an abort flag
// that every workgroup checks, so all waves leave the kernel.
#pragma once

#include "frontier.hpp"
#include "ops.hpp"

namespace gg {

struct GridBarrier {
    unsigned *arrive;   // [gridDim.x] last barrier epoch each workgroup reached
    unsigned *release;  // last epoch released by workgroup 0
    unsigned *abort;    // set when a wait exceeded the spin limit
    unsigned epoch;     // barriers passed so far (kept per lane, equal grid-wide)
};

constexpr long long kBarrierSpinLimit = 1ll << 24;  // ~seconds with s_sleep backoff

__device__ __forceinline__ unsigned ld_agent(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flag barrier: every workgroup publishes its arrival in its own word (no
// contended atomic), workgroup 0 polls all words in parallel and then
// publishes the release epoch that the others poll. One agent-scope release
// fence before arriving and one acquire fence after leaving; the polls are
// relaxed. Returns false when the barrier was aborted (the caller leaves).
__device__ __forceinline__ bool grid_sync(GridBarrier &b) {
    __shared__ unsigned s_abort;
    const unsigned ep = ++b.epoch;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_agent(&b.arrive[blockIdx.x], ep);
        s_abort = 0;
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        bool bad = false;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
            long long spins = 0;
            while (ld_agent(&b.arrive[i]) < ep) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kBarrierSpinLimit || ((spins & 255) == 0 && ld_agent(b.abort))) {
                    bad = true;
                    break;
                }
            }
            if (bad) break;
        }
        if (bad) { st_agent(b.abort, 1u); s_abort = 1; }
        __syncthreads();
        if (threadIdx.x == 0) st_agent(b.release, ep);
    } else if (threadIdx.x == 0) {
        long long spins = 0;
        while (ld_agent(b.release) < ep) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kBarrierSpinLimit || ((spins & 255) == 0 && ld_agent(b.abort))) {
                st_agent(b.abort, 1u);
                break;
            }
        }
    }
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (ld_agent(b.abort)) s_abort = 1;
    }
    __syncthreads();
    return s_abort == 0;
}

// STRICT inside a persistent kernel: the exclusive scan of the frontier's
// degrees, scan[0..size] (scan[size] = total), computed by the whole grid.
// Each workgroup sums the degrees of its contiguous slice into part[block];
// after a grid barrier every workgroup adds up the slices before its own and
// writes its slice's prefix sums, 256 at a time; a second barrier publishes
// the scan. Returns false when a barrier was aborted.
template <class Src>
__device__ bool grid_degree_scan(const DevGraph &g, const Src &src, long long *scan, long long *part,
                                 GridBarrier &bar) {
    __shared__ long long s_red[kBlock / kWave];
    __shared__ long long s_off;
    const int size = src.size;
    const int nb = (int)gridDim.x, b = (int)blockIdx.x, tid = (int)threadIdx.x;
    const int slice = (size + nb - 1) / nb;
    const int lo = min(size, b * slice), hi = min(size, lo + slice);
    long long sum = 0;
    for (int i = lo + tid; i < hi; i += kBlock) {
        const int u = src.get(i);
        sum += g.row_ptr[u + 1] - g.row_ptr[u];
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_red[tid / kWave] = sum;
    __syncthreads();
    if (tid == 0) {
        long long t = 0;
        for (int w = 0; w < kBlock / kWave; w++) t += s_red[w];
        part[b] = t;
    }
    if (!grid_sync(bar)) return false;
    // the slices before this one (and, for the last workgroup, all of them)
    long long before = 0, all = 0;
    for (int j = tid; j < nb; j += kBlock) {
        const long long v = part[j];
        if (j < b) before += v;
        all += v;
    }
    before = wave_sum(before);
    all = wave_sum(all);
    __syncthreads();
    if (lane_id() == 0) s_red[tid / kWave] = before;
    __syncthreads();
    if (tid == 0) {
        long long t = 0;
        for (int w = 0; w < kBlock / kWave; w++) t += s_red[w];
        s_off = t;
    }
    __syncthreads();
    if (lane_id() == 0) s_red[tid / kWave] = all;
    __syncthreads();
    if (b == nb - 1 && tid == 0) {
        long long t = 0;
        for (int w = 0; w < kBlock / kWave; w++) t += s_red[w];
        scan[size] = t;
    }
    long long off = s_off;
    for (int base = lo; base < hi; base += kBlock) {
        const int i = base + tid;
        long long d = 0;
        if (i < hi) {
            const int u = src.get(i);
            d = g.row_ptr[u + 1] - g.row_ptr[u];
        }
        const long long incl = wave_incl_scan64(d);
        __syncthreads();
        if (lane_id() == kWave - 1) s_red[tid / kWave] = incl;
        __syncthreads();
        long long wbefore = 0, tile = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; w++) {
            const long long v = s_red[w];
            if (w < tid / kWave) wbefore += v;
            tile += v;
        }
        if (i < hi) scan[i] = off + wbefore + incl - d;
        off += tile;
    }
    return grid_sync(bar);
}

// Co-resident grid for a persistent kernel: `per_cu` workgroups (of
// `threads` lanes) per compute unit, capped by the occupancy the kernel
// actually achieves; per_cu <= 0 asks for one workgroup per two units.
int fused_grid(const void *kernel, int per_cu, int num_cus, int threads = kBlock);
int fused_grid_for(const void *kernel, const Graph &G, int num_cus);

// Launch with the cooperative API (which refuses grids that cannot be
// co-resident).
void launch_cooperative(Ctx &c, const void *kernel, int blocks, void **args, int threads = kBlock);

// Allocate/zero the barrier words in the workspace for a grid of `blocks`.
GridBarrier prepare_barrier(Ctx &c, Workspace &ws, int blocks);
// Read the abort flag after the kernel; throws if the loop was aborted.
void check_barrier(Ctx &c, Workspace &ws);

}  // namespace gg
