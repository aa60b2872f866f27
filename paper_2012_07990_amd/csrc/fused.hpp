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

#include "ops.hpp"

namespace gg {

struct GridBarrier {
    unsigned *count;   // arrivals in the current phase
    unsigned *gen;     // phase number
    unsigned *abort;   // set when a wait exceeded the spin limit
};

constexpr long long kBarrierSpinLimit = 1ll << 25;  // ~seconds with s_sleep backoff

// Returns false when the barrier was aborted (the caller must then leave).
__device__ __forceinline__ bool grid_sync(const GridBarrier &b) {
    __shared__ unsigned s_abort;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nblocks = gridDim.x;
        const unsigned g = __hip_atomic_load(b.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(b.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(b.gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(b.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kBarrierSpinLimit) {
                    __hip_atomic_store(b.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if ((spins & 1023) == 0 &&
                    __hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        s_abort = __hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_abort == 0;
}

// Co-resident grid for a persistent kernel: `per_cu` workgroups per compute
// unit, capped by the occupancy the kernel actually achieves.
int fused_grid(const void *kernel, int per_cu, int num_cus);

// Launch with the cooperative API (which refuses grids that cannot be
// co-resident).
void launch_cooperative(Ctx &c, const void *kernel, int blocks, void **args);

// Allocate/zero the barrier words {count, gen, abort} in the workspace.
GridBarrier prepare_barrier(Ctx &c, Workspace &ws);
// Read the abort flag after the kernel; throws if the loop was aborted.
void check_barrier(Ctx &c, Workspace &ws);

}  // namespace gg
