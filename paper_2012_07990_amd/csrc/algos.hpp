// Algorithm drivers and schedule handling (declarations).
#pragma once

#include "ops.hpp"

namespace gg {

gg_schedule default_schedule();
gg_schedule preset_schedule(int algo, int preset);
// throws Error(GG_ERR_UNSUPPORTED_SCHEDULE / GG_ERR_INVALID_ARG) with the reason
void validate_schedule(const Graph &g, int algo, const gg_schedule &s);
size_t workspace_bytes(const Graph &g, int algo, int k);

void bfs_run(Graph &G, int32_t src, const gg_schedule &s, int32_t *depth, hipStream_t stream, gg_stats *st);
// the same on a caller-provided workspace (the graph's pool is not used)
void bfs_run_ws(Graph &G, Workspace &ws, int32_t src, const gg_schedule &s, int32_t *depth, hipStream_t stream,
                gg_stats *st);
void sssp_run(Graph &G, int32_t src, const gg_schedule &s, int32_t *dist, hipStream_t stream, gg_stats *st);
void cc_run(Graph &G, const gg_schedule &s, int32_t *label, hipStream_t stream, gg_stats *st);
void pr_run(Graph &G, const gg_schedule &s, float damping, int iters, uint32_t flags, float *rank,
            hipStream_t stream, gg_stats *st);
void bc_run(Graph &G, int32_t src, const gg_schedule &s, uint64_t *sigma, float *delta, hipStream_t stream,
            gg_stats *st);
void msbfs_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &s, int32_t *depth, hipStream_t stream,
               gg_stats *st);
// overflow_mask: when non-null, receives the sources whose distances overflow
// (instead of an exception)
// batched BFS as the unit-weight form of the batched delta-stepping loop
void msbfs_push_run(Graph &G, const int32_t *srcs, int k, int32_t *depth, hipStream_t stream, gg_stats *st);
void mssssp_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &s, int32_t *dist, hipStream_t stream,
                gg_stats *st, unsigned long long *overflow_mask);
size_t mssssp_work_bytes(const Graph &G, int k);
void msbc_run(Graph &G, const int32_t *srcs, int k, const gg_schedule &s, uint64_t *sigma, float *delta,
              hipStream_t stream, gg_stats *st);

gg_schedule autotune(Graph &G, int algo, double budget_s, const int32_t *probes, int nprobe, hipStream_t st,
                     double *best_ms);

// PULL EdgeBlocking layout build (cached on the graph); returns device milliseconds, 0 if cached
double pull_layout_prepare(Graph &G, int32_t seg_vertices, hipStream_t stream);
// EdgeBlocking preprocessing; returns milliseconds
double edgeblock_prepare(Ctx &c, Graph &G, int32_t seg_vertices);
// in-edges (transpose) of a directed graph, built once; no-op on symmetric graphs
void ensure_transpose(Ctx &c, Graph &G);
// true when a schedule may run a PULL step
inline bool schedule_pulls(const gg_schedule &s) {
    return s.s1.direction == GG_PULL || (s.hybrid && s.s2.direction == GG_PULL);
}

}  // namespace gg
