// Schedule defaults, presets and validation (SimpleGPUSchedule and
// HybridGPUSchedule tables of the Scheduling Language section).
#include <algorithm>
#include <string>

#include "algos.hpp"

namespace gg {

static gg_simple_schedule simple_default() {
    gg_simple_schedule s{};
    s.load_balance = GG_LB_VERTEX_BASED;
    s.edge_blocking = 0;
    s.blocking_size = 1 << 20;
    s.direction = GG_PUSH;
    s.pull_rep = GG_REP_BOOLMAP;
    s.frontier_creation = GG_CREATE_FUSED;
    s.dedup_enable = 1;
    s.dedup_type = GG_DEDUP_MONOTONIC_COUNTERS;
    s.delta = 1;
    s.kernel_fusion = 0;
    return s;
}

gg_schedule default_schedule() {
    gg_schedule s{};
    s.hybrid = 0;
    s.threshold = 0.05f;
    s.s1 = simple_default();
    s.s2 = simple_default();
    return s;
}

gg_schedule preset_schedule(int algo, int preset) {
    gg_schedule s = default_schedule();
    switch (preset) {
    case GG_PRESET_DEFAULT:
        break;
    case GG_PRESET_BFS_HYBRID:
        // the direction-optimising BFS schedule of the paper's GPU schedule figure
        s.hybrid = 1;
        s.s1.direction = GG_PUSH;
        s.s1.load_balance = GG_LB_VERTEX_BASED;
        s.s2 = s.s1;
        s.s2.direction = GG_PULL;
        s.s2.pull_rep = GG_REP_BITMAP;
        s.s2.dedup_enable = 0;
        s.s2.frontier_creation = GG_CREATE_UNFUSED_BITMAP;
        break;
    case GG_PRESET_ROAD_FUSED:
        s.s1.kernel_fusion = 1;
        s.s1.load_balance = GG_LB_CM;
        if (algo == GG_ALGO_SSSP) s.s1.delta = 64;
        break;
    case GG_PRESET_POWERLAW:
        s.s1.load_balance = GG_LB_ETWC;
        if (algo == GG_ALGO_BFS || algo == GG_ALGO_BC) {
            s.hybrid = 1;
            s.s2 = s.s1;
            s.s2.direction = GG_PULL;
            s.s2.pull_rep = GG_REP_BITMAP;
            s.s2.load_balance = GG_LB_VERTEX_BASED;
            s.s2.frontier_creation = GG_CREATE_UNFUSED_BITMAP;
            s.s2.dedup_enable = 0;
        }
        if (algo == GG_ALGO_PR) s.s1.load_balance = GG_LB_STRICT, s.s1.direction = GG_PULL;
        break;
    default:
        throw Error(GG_ERR_INVALID_ARG, "unknown preset");
    }
    return s;
}

static void bad(const std::string &m) { throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, m); }

static void check_simple(const Graph &g, int algo, const gg_simple_schedule &s, bool is_s2) {
    if (s.load_balance < 0 || s.load_balance > GG_LB_EDGE_ONLY) throw Error(GG_ERR_INVALID_ARG, "bad load_balance");
    if (s.direction != GG_PUSH && s.direction != GG_PULL) throw Error(GG_ERR_INVALID_ARG, "bad direction");
    if (s.pull_rep != GG_REP_BOOLMAP && s.pull_rep != GG_REP_BITMAP) throw Error(GG_ERR_INVALID_ARG, "bad pull_rep");
    if (s.frontier_creation < 0 || s.frontier_creation > GG_CREATE_UNFUSED_BITMAP)
        throw Error(GG_ERR_INVALID_ARG, "bad frontier_creation");
    if (s.dedup_type < 0 || s.dedup_type > GG_DEDUP_BOOLMAP) throw Error(GG_ERR_INVALID_ARG, "bad dedup_type");
    if (s.delta < 1) throw Error(GG_ERR_INVALID_ARG, "delta must be >= 1");
    if (s.edge_blocking && s.blocking_size < 1) throw Error(GG_ERR_INVALID_ARG, "blocking_size must be >= 1");
    // PULL reads in-edges: the CSR itself on a symmetric graph, else its
    // transpose (built once per graph on first use)
    // EdgeBlocking applies only when every edge is processed (the edge
    // processing algorithm's note): the topology-driven PageRank sweep.
    if (s.edge_blocking) {
        if (algo != GG_ALGO_PR && algo != GG_ALGO_CC && algo != GG_ALGO_SSSP)
            bad("EdgeBlocking applies only to all-edges operators (PageRank, the CC hook sweep, SSSP's EDGE_ONLY "
                "rounds)");
        if (algo == GG_ALGO_SSSP && (s.load_balance != GG_LB_EDGE_ONLY || s.direction != GG_PUSH || s.kernel_fusion))
            bad("SSSP EdgeBlocking runs unfused EDGE_ONLY rounds over destination segments");
        const bool push_eb = s.load_balance == GG_LB_EDGE_ONLY && s.direction == GG_PUSH;
        const bool pull_eb = s.load_balance == GG_LB_STRICT && s.direction == GG_PULL;
        if (algo == GG_ALGO_CC) {
            if (!push_eb || s.kernel_fusion)
                bad("CC EdgeBlocking runs the unfused EDGE_ONLY sweep over destination segments");
            if (((long long)g.n + s.blocking_size - 1) / s.blocking_size > 64)
                bad("CC EdgeBlocking supports at most 64 segments (blocking_size >= n / 64)");
        } else if (!push_eb && !pull_eb) {
            bad("EdgeBlocking runs EDGE_ONLY in the PUSH direction (destination segments) or STRICT in the "
                "PULL direction (source segments)");
        }
    }
    switch (algo) {
    case GG_ALGO_BFS:
    case GG_ALGO_BC:
        if (s.direction == GG_PULL && s.load_balance != GG_LB_VERTEX_BASED)
            bad("PULL traversal runs VERTEX_BASED (one lane per destination)");
        break;
    case GG_ALGO_SSSP:
        if (s.direction == GG_PULL) bad("SSSP runs PUSH only");
        break;
    case GG_ALGO_CC:
        if (s.direction == GG_PULL) bad("CC runs PUSH only");
        break;
    case GG_ALGO_PR:
        if (s.direction == GG_PULL && s.load_balance != GG_LB_VERTEX_BASED && s.load_balance != GG_LB_WM &&
            s.load_balance != GG_LB_STRICT && s.load_balance != GG_LB_ETWC)
            bad("PageRank PULL supports VERTEX_BASED, WM, ETWC and STRICT");
        if (s.direction == GG_PUSH && s.load_balance != GG_LB_EDGE_ONLY)
            bad("PageRank PUSH runs EDGE_ONLY (every edge, every round)");
        break;
    default:
        throw Error(GG_ERR_INVALID_ARG, "unknown algorithm");
    }
    if (s.kernel_fusion && !is_s2) {
        if (algo != GG_ALGO_BFS && algo != GG_ALGO_SSSP && algo != GG_ALGO_CC)
            bad("kernel fusion is available for BFS, SSSP and CC loops");
        if (s.load_balance != GG_LB_VERTEX_BASED && s.load_balance != GG_LB_WM && s.load_balance != GG_LB_CM &&
            s.load_balance != GG_LB_ETWC && s.load_balance != GG_LB_STRICT)
            bad("kernel fusion supports VERTEX_BASED, WM, CM, ETWC and STRICT (device-side load balancers; "
                "STRICT's degree scan runs inside the persistent grid)");
        if (s.frontier_creation != GG_CREATE_FUSED) bad("kernel fusion keeps the frontier as a queue (FUSED creation)");
        if (algo != GG_ALGO_BFS && s.direction == GG_PULL) bad("fused loops run PUSH");
    }
}

void validate_schedule(const Graph &g, int algo, const gg_schedule &s) {
    check_simple(g, algo, s.s1, false);
    if (s.hybrid) {
        if (!(s.threshold > 0.f && s.threshold <= 1.f)) throw Error(GG_ERR_INVALID_ARG, "threshold must be in (0, 1]");
        check_simple(g, algo, s.s2, true);
        if (algo != GG_ALGO_BFS && algo != GG_ALGO_BC && algo != GG_ALGO_SSSP)
            bad("hybrid schedules apply to BFS, BC (push/pull) and SSSP (sparse/dense rounds)");
        if (algo == GG_ALGO_SSSP && s.s1.kernel_fusion) bad("a hybrid SSSP loop runs unfused");
        if (s.s1.kernel_fusion && s.s2.direction == GG_PUSH && s.s2.load_balance != s.s1.load_balance)
            bad("a fused hybrid loop pushes with s1's load balancer");
        if (s.s1.kernel_fusion && algo != GG_ALGO_BFS) bad("fused hybrid loops are available for BFS");
    }
}

size_t workspace_bytes(const Graph &g, int algo, int k) {
    // an upper bound of what one call may add to a workspace: pooled
    // workspaces are shared by every schedule and algorithm, so the frontier
    // part is the union over schedules (queues 8n, boolmaps 2n, bitmaps n/4,
    // tags 4n, dedup maps 1.125n, STRICT degree scan 8n, TWC tiers 12n,
    // EDGE_ONLY membership n, small counters)
    const size_t n = (size_t)g.n + 256, m = (size_t)g.m;
    size_t b = 37 * n + 65536;
    switch (algo) {
    case GG_ALGO_SSSP: b += 3 * n * 4; break;                   // far queues, far tags
    case GG_ALGO_PR: b += 24 * n + m / 16 + 65536; break;        // contributions, fp64 sums, LDS-cache tables, chunk heads/tails
    case GG_ALGO_BC: b += 4 * n + 2 * n * 8 + n; break;          // depth, delta and t, one-byte depths
    default: break;
    }
    if (k > 1) {
        b += 3 * n * 8;  // multi-source masks
        if (algo == GG_ALGO_BFS) b += (size_t)k * n * 4;  // per-source depths, vertex-major
        // per group of up to 16 sources: sigma, delta and t (8 B each) and depth (4 B)
        if (algo == GG_ALGO_BC) b += (size_t)std::min(k, 16) * n * 28;
        if (algo == GG_ALGO_SSSP) b += (size_t)k * n * 4 + 2 * n * 4;
    }
    return b;
}

}  // namespace gg
