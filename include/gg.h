/*
 * gg.h -- C ABI of the MI355X (gfx950) frontier-traversal library.
 *
 * The library runs the frontier-driven edge traversal of "Compilation
 * Techniques for Graph Algorithms on GPUs" (Brahmakshatriya et al., CGO 2021):
 * edges.from(frontier).to(filter).apply(update), the operator of the paper's
 * Algorithm Language section (BFS program figure), under the schedule
 * choices of its Scheduling Language section (SimpleGPUSchedule and
 * HybridGPUSchedule tables): load balancing, push/pull direction, frontier
 * representation and creation, deduplication, delta-stepping buckets,
 * EdgeBlocking and kernel fusion.
 *
 * Conventions for every entry point:
 *   - Every call returns a gg_status; no C++ exception crosses this ABI.
 *     On failure gg_last_error() returns a thread-local message.
 *   - Graph arrays passed to gg_graph_create_csr are host pointers unless
 *     GG_INPUT_DEVICE is set. The library copies them: the caller keeps
 *     ownership of its arrays.
 *   - Output arrays (depth, dist, label, rank, sigma, delta) are caller-owned
 *     DEVICE memory (e.g. a torch tensor's data_ptr) of the stated length.
 *   - Calls are stream-ordered on `stream` (0 = the null stream) and return
 *     once the result is complete on that stream.
 *   - A graph is immutable after creation apart from cached derived layouts;
 *     queries on one graph may run concurrently on distinct streams (each call
 *     takes a private workspace from the graph's mutex-protected pool).
 *   - The library allocates device memory only for the graph copy, derived
 *     layouts and cached workspaces; everything is released by
 *     gg_graph_destroy.
 */
#ifndef GG_H
#define GG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without pulling in HIP headers */
typedef struct ihipStream_t *gg_stream_t;

typedef enum {
    GG_OK = 0,
    GG_ERR_INVALID_ARG = 1,
    GG_ERR_OUT_OF_MEMORY = 2,
    GG_ERR_DEVICE = 3,               /* a HIP call failed; message keeps hipError text */
    GG_ERR_UNSUPPORTED_SCHEDULE = 4, /* combination the operator cannot run */
    GG_ERR_OVERFLOW = 5,             /* result not representable (SSSP dist, BC sigma) */
    GG_ERR_ADMISSION = 6,            /* serving: query can never fit the memory budget */
    GG_ERR_NOT_FOUND = 7,            /* serving: unknown ticket */
    GG_ERR_NOT_READY = 8             /* serving: result not complete yet */
} gg_status;

/* ---- algorithms ---------------------------------------------------------- */
typedef enum { GG_ALGO_BFS = 0, GG_ALGO_SSSP = 1, GG_ALGO_CC = 2, GG_ALGO_PR = 3, GG_ALGO_BC = 4 } gg_algo;

/* ---- schedule (SimpleGPUSchedule / HybridGPUSchedule tables) --------------- */
/* configLoadBalance: work-to-thread mapping of the active edges
   (GPU Optimization Space section, "Load Balancing"; ETWC algorithm). */
typedef enum {
    GG_LB_VERTEX_BASED = 0, /* one lane per active vertex */
    GG_LB_WM = 1,           /* active vertices split evenly over wavefronts */
    GG_LB_CM = 2,           /* active vertices split evenly over workgroups */
    GG_LB_STRICT = 3,       /* every lane gets the same number of edges */
    GG_LB_TWC = 4,          /* grid-wide degree binning into lane/wave/workgroup tiers */
    GG_LB_ETWC = 5,         /* per-workgroup chunking into workgroup/wave/lane stages */
    GG_LB_EDGE_ONLY = 6     /* edge-parallel over all edges (COO) */
} gg_load_balance;

/* configDirection */
typedef enum { GG_PUSH = 0, GG_PULL = 1 } gg_direction;
/* frontier representation read by PULL (configDirection's optional argument) */
typedef enum { GG_REP_BOOLMAP = 0, GG_REP_BITMAP = 1 } gg_frontier_rep;
/* configFrontierCreation */
typedef enum { GG_CREATE_FUSED = 0, GG_CREATE_UNFUSED_BOOLMAP = 1, GG_CREATE_UNFUSED_BITMAP = 2 } gg_frontier_creation;
/* configDeduplication strategy */
typedef enum { GG_DEDUP_MONOTONIC_COUNTERS = 0, GG_DEDUP_BITMAP = 1, GG_DEDUP_BOOLMAP = 2 } gg_dedup_type;

typedef struct {
    int32_t load_balance;      /* gg_load_balance, default VERTEX_BASED */
    int32_t edge_blocking;     /* 0/1: EdgeBlocking (all-edges operators only) */
    int32_t blocking_size;     /* vertices per EdgeBlocking segment, default 2^20 */
    int32_t direction;         /* gg_direction, default PUSH */
    int32_t pull_rep;          /* gg_frontier_rep, default BOOLMAP */
    int32_t frontier_creation; /* gg_frontier_creation, default FUSED */
    int32_t dedup_enable;      /* 0/1, default 1 */
    int32_t dedup_type;        /* gg_dedup_type, default MONOTONIC_COUNTERS */
    int32_t delta;             /* configDelta: bucket width for SSSP, default 1 */
    int32_t kernel_fusion;     /* configKernelFusion: 0/1, default 0 (unfused, as the
                                  paper's default PUSH schedule and fusion baseline) */
} gg_simple_schedule;

/* HybridGPUSchedule with the INPUT_VERTEXSET_SIZE criterion: an iteration
   runs s2 when |input frontier| > threshold * n, else s1. With hybrid == 0
   only s1 is used. Kernel fusion of the loop is taken from s1. */
typedef struct {
    int32_t hybrid;
    float threshold;
    gg_simple_schedule s1;
    gg_simple_schedule s2;
} gg_schedule;

typedef enum {
    GG_PRESET_DEFAULT = 0,     /* PUSH, VERTEX_BASED, FUSED, dedup monotonic */
    GG_PRESET_BFS_HYBRID = 1,  /* the paper's direction-optimising BFS schedule */
    GG_PRESET_ROAD_FUSED = 2,  /* PUSH, fused loop (high-diameter graphs) */
    GG_PRESET_POWERLAW = 3     /* ETWC push / hybrid for power-law graphs */
} gg_preset;

/* ---- statistics ------------------------------------------------------------ */
#define GG_STATS_COUNT_EDGES 1u  /* request device counters of examined edges */
#define GG_STATS_TIME_KERNELS 2u /* time the main edge-traversal kernel with HIP events */
typedef struct {
    uint32_t flags;            /* in: GG_STATS_* requests */
    int32_t iterations;        /* levels / rounds / bucket phases executed */
    int32_t push_iterations;   /* iterations run with a PUSH schedule */
    int32_t pull_iterations;   /* iterations run with a PULL schedule */
    int32_t launches;          /* kernels launched by the call */
    int32_t buckets;           /* SSSP: non-empty buckets processed */
    int32_t fused;             /* 1 if the loop ran as one persistent launch */
    int64_t edges_examined;    /* with GG_STATS_COUNT_EDGES */
    int64_t vertices_processed;/* with GG_STATS_COUNT_EDGES: sum of frontier sizes */
    double device_ms;          /* wall time of the call's device work */
    double kernel_ms;          /* with GG_STATS_TIME_KERNELS: summed event time of the
                                  main edge-traversal kernel's launches */
    int32_t kernel_launches;   /* with GG_STATS_TIME_KERNELS: launches of that kernel */
    char kernel_name[44];      /* with GG_STATS_TIME_KERNELS: that kernel's name */
} gg_stats;

/* ---- errors ------------------------------------------------------------------ */
const char *gg_status_string(gg_status s);
/* Thread-local message describing the last failure on this thread ("" if none). */
const char *gg_last_error(void);
/* Library version string. */
const char *gg_version(void);

/* ---- graph ----------------------------------------------------------------------- */
typedef struct gg_graph gg_graph;

#define GG_INPUT_DEVICE 1u /* row_ptr/col/w are device pointers */
#define GG_VALIDATE 2u     /* O(m) check: row_ptr[0]=0, monotone, row_ptr[n]=m,
                              0<=col<n, rows strictly ascending, no self-loops */
#define GG_SYMMETRIC 4u    /* caller asserts (u,v) in E <=> (v,u) in E; required by
                              CC, the batched BFS/BC forms and serving. Without it
                              the CSR rows are out-edges: PULL steps read the
                              graph's transpose (in-rows, sources ascending), built
                              on the host once, on first use */

/*
 * Build a device-resident CSR graph (the `load` of the paper's BFS program).
 * n >= 1 vertices, m directed entries (0 <= m < 2^31); row_ptr[n+1], col[m]
 * int32; w[m] uint32 edge weights or NULL (SSSP requires weights in
 * [1, 2^31/n]). The arrays are copied. Errors: GG_ERR_INVALID_ARG for bad
 * sizes/pointers or a failed GG_VALIDATE check, GG_ERR_OUT_OF_MEMORY,
 * GG_ERR_DEVICE.
 */
gg_status gg_graph_create_csr(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                              const uint32_t *w, uint32_t flags, gg_stream_t stream,
                              gg_graph **out);
/* Frees the graph, its derived layouts and cached workspaces. NULL is a no-op. */
gg_status gg_graph_destroy(gg_graph *g);
gg_status gg_graph_info(const gg_graph *g, int32_t *n, int64_t *m, int32_t *has_weights,
                        int32_t *symmetric);

/*
 * EdgeBlocking preprocessing (GPU-Specific Optimizations section, Algorithm
 * for preprocessing the input graph): the COO edge list is counted per
 * destination segment floor(dst / seg_vertices), an exclusive prefix sum
 * gives each segment's start, and a stable scatter writes the blocked COO.
 * Owned by the graph, cached per seg_vertices (idempotent). prep_ms (may be
 * NULL) receives the preprocessing time.
 */
gg_status gg_graph_prepare_edgeblocking(gg_graph *g, int32_t seg_vertices, gg_stream_t stream,
                                        double *prep_ms);
/*
 * PULL EdgeBlocking layout (not in the paper; the gather-side counterpart of
 * the paper's EdgeBlocking, used by PageRank PULL + STRICT with
 * edge_blocking set): the in-edge CSR (the graph's own when symmetric, else
 * its transpose) split by source segment [s*seg_vertices,
 * (s+1)*seg_vertices) into S segment CSRs (rows keep their order) plus the
 * STRICT chunk-to-row partition of each. Owned by the graph, cached per
 * seg_vertices (a later gg_pagerank with that width reuses it). prep_ms (may
 * be NULL) receives the build time on the device (0 when it was cached).
 */
gg_status gg_graph_prepare_pull_blocking(gg_graph *g, int32_t seg_vertices, gg_stream_t stream, double *prep_ms);
/*
 * Copy the blocked COO built by gg_graph_prepare_edgeblocking into caller
 * device buffers src_dev[m], dst_dev[m] and host seg_start[S+1]
 * (S = ceil(n / seg_vertices)); segment s holds entries [seg_start[s],
 * seg_start[s+1]). GG_ERR_INVALID_ARG if that blocking was not prepared.
 */
gg_status gg_graph_edgeblocking_export(const gg_graph *g, int32_t seg_vertices, int32_t *src_dev,
                                       int32_t *dst_dev, int64_t *seg_start_host,
                                       gg_stream_t stream);

/* ---- schedules ---------------------------------------------------------------------- */
/* Defaults of the SimpleGPUSchedule table; fusion defaults to disabled. */
gg_status gg_schedule_default(gg_schedule *s);
gg_status gg_schedule_preset(int32_t algo, int32_t preset, gg_schedule *s);
/* GG_OK if `algo` can run `s` on `g`, else GG_ERR_UNSUPPORTED_SCHEDULE or
   GG_ERR_INVALID_ARG with the reason in gg_last_error(). */
gg_status gg_schedule_validate(const gg_graph *g, int32_t algo, const gg_schedule *s);

/* ---- algorithms (Evaluation section, "Algorithms") ------------------------------------- */
/*
 * BFS from src: depth_dev[n] int32 receives the hop count, -1 when
 * unreachable (the depth is the unique part of the paper's parent-array BFS).
 * A PUSH round claims each vertex with one CAS, so its output queue holds no
 * duplicates: the schedule's deduplication setting changes nothing and is
 * not applied.
 */
gg_status gg_bfs(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *depth_dev,
                 gg_stream_t stream, gg_stats *stats);
/*
 * gg_bfs for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * BFS and outputs as gg_bfs, with its workspace carved from a fixed 40 MiB
 * device array that each GPU holds until the process ends. It calls no
 * hipMalloc, hipFree or allocating library routine. Limits: n <= 1,048,576
 * (else GG_ERR_INVALID_ARG); GG_ERR_UNSUPPORTED_SCHEDULE for EDGE_ONLY
 * (it needs the graph's COO array) and for PULL on a directed graph whose
 * transpose has not been built yet (one PULL query through gg_bfs builds
 * it); no stats. The graph must live on the current device. Every call on
 * one GPU shares that GPU's array and leaves its contents behind (whatever
 * must start at zero is cleared by each call): calls that overlap on one
 * GPU race.
 */
gg_status gg_bfs_noalloc(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *depth_dev,
                         gg_stream_t stream);
/*
 * Delta-stepping SSSP from src with the schedule's delta (priority-queue
 * schedule, configDelta): dist_dev[n] int32, INT32_MAX when unreachable.
 * Requires weights. GG_ERR_OVERFLOW when a distance would exceed INT32_MAX-1.
 * A hybrid schedule (HybridGPUSchedule with INPUT_VERTEXSET_SIZE) runs s2 in
 * the relaxation rounds whose input frontier holds more than threshold * n
 * vertices and s1 in the others; s1 fixes delta and must be unfused. s2 may
 * be EDGE_ONLY with edge_blocking: such a round relaxes every edge whose
 * source is in the frontier, over the EdgeBlocked COO (destination segments
 * of blocking_size vertices, built once per width with the edges' weights,
 * as gg_graph_prepare_edgeblocking does), one launch per segment.
 */
gg_status gg_sssp(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *dist_dev,
                  gg_stream_t stream, gg_stats *stats);
/* Connected components (hooking + shortcutting): label_dev[n] int32 = the
   smallest vertex id of the component. Requires GG_SYMMETRIC. EDGE_ONLY
   sweeps every undirected edge once per round; with edge_blocking set the
   sweep runs over that pair list grouped by the segment floor(v /
   blocking_size) of the larger endpoint (the EdgeBlocking preprocessing
   applied to this all-edges operator; built on the device once per width
   and owned by the graph), one launch per segment; at most 64 segments
   (GG_ERR_UNSUPPORTED_SCHEDULE otherwise). */
gg_status gg_cc(gg_graph *g, const gg_schedule *s, int32_t *label_dev, gg_stream_t stream,
                gg_stats *stats);

#define GG_PR_NO_DANGLING 1u /* drop the mass of zero-degree vertices */
/* PULL STRICT only: gather every source's contribution from global memory
   instead of keeping the highest-degree sources of each segment in LDS.
   The results are bit-identical either way (same values, same order). */
#define GG_PR_NO_LDS_CACHE 2u
/* PageRank, fp32: `iters` power-iteration rounds from 1/n with damping
   `damping`: rank'(v) = (1-d)/n + d * (sum over in-neighbours u of
   rank(u)/outdeg(u) + D/n), D = the rank of vertices without out-edges
   (dropped with GG_PR_NO_DANGLING). rank_dev[n] float. Directed graphs:
   PULL sums over the transpose, PUSH scatters along out-edges. */
gg_status gg_pagerank(gg_graph *g, const gg_schedule *s, float damping, int32_t iters,
                      uint32_t flags, float *rank_dev, gg_stream_t stream, gg_stats *stats);
/* Single-source Brandes betweenness: sigma_dev[n] uint64 shortest-path
   counts, delta_dev[n] float dependencies (delta[src] = 0). GG_ERR_OVERFLOW
   when a path count would exceed 2^64-1. Directed graphs: shortest paths
   follow out-edges (PULL forward steps read the transpose). */
gg_status gg_bc(gg_graph *g, int32_t src, const gg_schedule *s, uint64_t *sigma_dev,
                float *delta_dev, gg_stream_t stream, gg_stats *stats);

/* ---- batched multi-source --------------------------------------------------------------- */
/* k <= 64 sources (host array) in one batched traversal; depth_dev is k x n
   row-major. The schedule picks the form (configDirection): PUSH without a
   hybrid switch runs a sparse-queue loop in one persistent launch (one grid
   barrier per level, work proportional to the frontier: high-diameter
   graphs); PULL or hybrid runs a bit-packed PULL sweep per level (every
   edge's column and frontier word read once for all sources: low-diameter
   graphs). Bit-identical to k gg_bfs calls. */
gg_status gg_bfs_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s,
                       int32_t *depth_dev, gg_stream_t stream, gg_stats *stats);
/* k <= 64 delta-stepping SSSP sources (host array) sharing one bucket loop
   in one persistent launch (configDelta of the Scheduling Language section;
   Kernel Fusion across Iterations): dist_dev is k x n row-major int32,
   unreached = INT32_MAX. The schedule contributes s1.delta (>= 1) only; the
   batch always runs fused. Requires weights and max degree < 2^25.
   GG_ERR_OVERFLOW when any source's distance would exceed INT32_MAX-1.
   Bit-identical to k gg_sssp calls. */
gg_status gg_sssp_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s,
                        int32_t *dist_dev, gg_stream_t stream, gg_stats *stats);
/* k <= 64 BC sources; sigma_dev / delta_dev are k x n row-major.
   Bit-identical to k gg_bc calls. */
gg_status gg_bc_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s,
                      uint64_t *sigma_dev, float *delta_dev, gg_stream_t stream, gg_stats *stats);

/*
 * Autotuner (Auto-tuning subsection of the Compiler Implementation section):
 * successive halving over the valid schedules of `algo` on g (load balancing,
 * direction / hybrid threshold, frontier representation and creation,
 * fusion, delta, EdgeBlocking width), timed on the probe sources (host array
 * of nprobe ids; unused by CC and PR) within budget_s seconds of wall time.
 * The fastest schedule is written to *out (its time in *best_ms, may be
 * NULL) and cached on the graph: with budget_s <= 0 a cached winner is
 * returned without timing. Timing-based, so repeated tuning may differ.
 */
gg_status gg_autotune(gg_graph *g, int32_t algo, double budget_s, const int32_t *probe_srcs, int32_t nprobe,
                      gg_stream_t stream, gg_schedule *out, double *best_ms);

/* The tuned-schedule cache of g (the one gg_autotune fills and, with
   budget_s <= 0, returns). gg_tuned_set seeds it with a schedule found
   earlier, e.g. one stored under the graph's checksum by a previous process;
   the schedule is validated for `algo` on g (GG_ERR_UNSUPPORTED_SCHEDULE
   otherwise) and `ms` is kept as its measured time. gg_tuned_get copies the
   cached schedule of `algo` to *out (and its time to *ms, may be NULL);
   GG_ERR_NOT_FOUND when nothing is cached. Host-only: no device work. */
gg_status gg_tuned_set(gg_graph *g, int32_t algo, const gg_schedule *s, double ms);
gg_status gg_tuned_get(gg_graph *g, int32_t algo, gg_schedule *out, double *ms);

/* Device bytes of workspace a query of `algo` with k sources needs on g. */
gg_status gg_workspace_bytes(const gg_graph *g, int32_t algo, int32_t k, size_t *out);

/* ---- serving ------------------------------------------------------------------------- */
/*
 * A request loop over device-resident graphs. Queries are admitted by device-
 * memory footprint (a query that could never fit the budget is refused with
 * GG_ERR_ADMISSION at submission; others wait until memory frees up) and are
 * batched continuously: whenever a worker stream is free it takes the oldest
 * pending query together with every pending query of the same graph and
 * algorithm (BFS up to 64 per bit-packed launch, BC up to 16; SSSP, CC and
 * PageRank one per launch). Worker streams run concurrently. A query's result
 * stays on the device, charged to the budget, until it is polled. Batched
 * results are bit-identical to single-source calls, so a query's result does
 * not depend on what it was batched with. A query whose schedule is a
 * persistent (fused) loop runs alone on the device (other batches wait).
 */
typedef struct gg_server gg_server;

typedef struct {
    int64_t ticket;
    int32_t status;      /* the query's gg_status */
    int32_t graph_id, algo, src;
    int32_t batch_size;  /* queries that shared its launch */
    double queue_ms;     /* arrival -> start of its batch */
    double latency_ms;   /* arrival -> result complete on the device */
} gg_result;

typedef struct {
    int64_t submitted, completed, collected, rejected, batches;
    int32_t max_batch;
    size_t bytes_in_use; /* running batches' workspaces + uncollected results */
    size_t bytes_peak;   /* peak of bytes_in_use + bytes_idle at batch admission */
    double busy_ms;      /* summed wall time of executed batches */
    size_t bytes_idle;   /* held between batches: pooled workspaces, derived layouts */
    int64_t trims;       /* admissions that freed pooled workspaces first */
} gg_serve_stats;

#define GG_OUT_DEVICE 0u  /* `out` is device memory */
#define GG_OUT_HOST 1u    /* `out` is host memory */
#define GG_OUT_DISCARD 2u /* drop the result */

/* hbm_budget: device bytes the server may hold for workspaces and results;
   nstreams: concurrent worker streams (1..16). */
gg_status gg_server_create(size_t hbm_budget, int32_t nstreams, gg_server **out);
/* Register a symmetric graph (caller keeps ownership; it must outlive the
   server). All graphs are added before the first query. */
gg_status gg_server_add_graph(gg_server *srv, gg_graph *g, int32_t *gid);
/* Override the schedule used for (graph, algorithm); default: the graph's
   tuned schedule when it is not fused, else the power-law preset. */
gg_status gg_server_set_schedule(gg_server *srv, int32_t gid, int32_t algo, const gg_schedule *s);
gg_status gg_server_submit(gg_server *srv, int32_t gid, int32_t algo, int32_t src, int64_t *ticket);
/* Non-blocking: GG_ERR_NOT_READY while running. When done, copies the result
   (BFS/SSSP/CC: int32[n]; PR: float[n]; BC: uint64[n] sigma then float[n]
   delta) to `out` per `flags` (NULL or GG_OUT_DISCARD drops it), releases it
   and returns the query's status. GG_ERR_NOT_FOUND for unknown tickets. */
gg_status gg_server_poll(gg_server *srv, int64_t ticket, void *out, uint32_t flags, gg_result *res);
/* As poll, blocking up to timeout_s seconds (< 0: no limit). */
gg_status gg_server_wait(gg_server *srv, int64_t ticket, double timeout_s, void *out, uint32_t flags,
                         gg_result *res);
gg_status gg_server_stats(gg_server *srv, gg_serve_stats *out);
/* Runs the pending queries to completion, frees uncollected results. */
gg_status gg_server_destroy(gg_server *srv);

/* ---- CPU backend and CPU-or-GPU placement ------------------------------------------------ */
/*
 * The same algorithms on the host with a pool of threads (the paper's
 * Evaluation compares its CPU and GPU backends on one algorithm
 * specification; delta-stepping on road graphs ran faster on the CPU).
 * gg_cpu_graph_create copies a host CSR (GG_SYMMETRIC and GG_VALIDATE as for
 * gg_graph_create_csr; GG_INPUT_DEVICE is refused). Outputs are host arrays of
 * n entries with the GPU entry points' meanings; nthreads <= 0 uses every
 * hardware thread. Depths, distances, labels and path counts equal the GPU's
 * bit for bit; PageRank (fp32) and BC dependencies agree within the GPU's
 * tolerances, and no result depends on the thread count. Errors as for the
 * GPU entry points, with the message in gg_last_error().
 */
typedef struct gg_cpu_graph gg_cpu_graph;
gg_status gg_cpu_graph_create(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                              const uint32_t *w, uint32_t flags, gg_cpu_graph **out);
gg_status gg_cpu_graph_destroy(gg_cpu_graph *g);
gg_status gg_cpu_bfs(gg_cpu_graph *g, int32_t src, int32_t nthreads, int32_t *depth);
gg_status gg_cpu_sssp(gg_cpu_graph *g, int32_t src, int32_t delta, int32_t nthreads, int32_t *dist);
gg_status gg_cpu_cc(gg_cpu_graph *g, int32_t nthreads, int32_t *label);
gg_status gg_cpu_pagerank(gg_cpu_graph *g, float damping, int32_t iters, uint32_t flags, int32_t nthreads,
                          float *rank);
gg_status gg_cpu_bc(gg_cpu_graph *g, int32_t src, int32_t nthreads, uint64_t *sigma, float *delta);

#define GG_TARGET_GPU 0
#define GG_TARGET_CPU 1
/*
 * Place `algo` on the CPU or the GPU for this graph: the query (from src,
 * under schedule s on the GPU, with s's delta on the CPU; PageRank 20
 * rounds, d = 0.85) runs once to warm up and once timed on each backend, and
 * the faster target is returned (and cached on g; gg_placement_get reads it).
 * g and cg must hold the same graph. gpu_ms / cpu_ms (may be NULL) receive
 * the timed runs.
 */
gg_status gg_place(gg_graph *g, gg_cpu_graph *cg, int32_t algo, const gg_schedule *s, int32_t src,
                   int32_t nthreads, gg_stream_t stream, int32_t *target, double *gpu_ms, double *cpu_ms);
/* The cached placement of `algo` (GG_ERR_NOT_FOUND before gg_place). */
gg_status gg_placement_get(const gg_graph *g, int32_t algo, int32_t *target);

#ifdef __cplusplus
}
#endif
#endif /* GG_H */
