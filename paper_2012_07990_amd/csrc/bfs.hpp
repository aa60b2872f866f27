// BFS edge functors and driver entry points.
#pragma once

#include "ops.hpp"

namespace gg {

// PUSH update: claim an unvisited destination with a compare-and-swap of its
// level (the atomic form of the BFS program's updateEdge under toFilter).
struct BfsPush {
    int32_t *depth;
    int next;
    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    // load() issues the edge's reads (no side effects), apply() its updates;
    // load balancers batch the loads of several edges before applying them
    using Pre = int;
    __device__ __forceinline__ Pre load(int, int v, int) const { return depth[v]; }
    // two-phase form: the CAS's old value, else the loaded depth (a value the
    // compiler cannot fold, so the result test stays out of the CAS's branch)
    using Tok = int;
    __device__ __forceinline__ Tok issue(int, int v, int, Pre dv, bool ok) const {
        int r = dv;
        if (ok && dv < 0) r = atomic_cas_i32(&depth[v], -1, next);  // filter: a stale read only costs a failed CAS
        return r;
    }
    __device__ __forceinline__ int finish(int, int v, int, Pre, bool ok, Tok r) const {
        return ok && r == -1 ? v : -1;
    }
    __device__ __forceinline__ int apply(int u, int v, int e, Pre dv) const {
        return finish(u, v, e, dv, true, issue(u, v, e, dv, true));
    }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, load(u, v, e)); }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};


void bfs_fused(Ctx &c, Graph &G, Workspace &ws, int32_t src, const gg_schedule &s, int32_t *depth,
               gg_stats *st);

}  // namespace gg
