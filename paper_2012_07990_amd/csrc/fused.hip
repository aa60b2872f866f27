// Host helpers for persistent (fused) kernels: co-resident grid sizing,
// cooperative launch and the grid barrier's state.
#include "fused.hpp"

namespace gg {

int fused_grid(const void *kernel, int per_cu, int num_cus, int threads) {
    int occ = 0;
    GG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0));
    require(occ >= 1, GG_ERR_DEVICE, "fused kernel cannot be resident on a compute unit");
    if (per_cu <= 0) return num_cus / 2 > 0 ? num_cus / 2 : 1;  // half a workgroup per CU
    const int per = per_cu < occ ? per_cu : occ;
    return per * num_cus;
}

// Persistent grid size for a graph: every grid barrier pays an agent-scope
// release and acquire per workgroup (measured ~12 us per barrier at 512
// workgroups, ~5 us at 128, ~3 us at 32), so sparse, high-diameter graphs --
// frontiers of a few thousand vertices, thousands of rounds -- get one
// workgroup per eight compute units (on a 2048 x 2048 grid, fused BFS and
// SSSP rounds measured 11.5 us at 32 workgroups, 14.4 at 128, 19.9 at 512);
// dense graphs keep two per compute unit for parallelism.
int fused_grid_for(const void *kernel, const Graph &G, int num_cus) {
    const bool sparse = G.m < 8ll * (long long)G.n;
    if (sparse) {
        fused_grid(kernel, 1, num_cus);  // checks that the kernel can be resident
        return num_cus / 8 > 0 ? num_cus / 8 : 1;
    }
    return fused_grid(kernel, 2, num_cus);
}

void launch_cooperative(Ctx &c, const void *kernel, int blocks, void **args, int threads) {
    GG_HIP(hipLaunchCooperativeKernel(kernel, dim3(blocks), dim3(threads), args, 0, c.s));
    c.launches++;
}

GridBarrier prepare_barrier(Ctx &c, Workspace &ws, int blocks) {
    ws.barrier.ensure((size_t)blocks + 4);
    fill_i32(c, reinterpret_cast<int32_t *>(ws.barrier.p), blocks + 4, 0);
    return GridBarrier{ws.barrier.p + 4, ws.barrier.p + 1, ws.barrier.p + 2, 0u};
}

void check_barrier(Ctx &c, Workspace &ws) {
    unsigned v[4];
    GG_HIP(hipMemcpyAsync(v, ws.barrier.p, sizeof(v), hipMemcpyDeviceToHost, c.s));  // {-, release, abort, -}
    GG_HIP(hipStreamSynchronize(c.s));
    require(v[2] == 0, GG_ERR_DEVICE, "fused kernel aborted: a grid barrier wait exceeded its limit");
}

}  // namespace gg
