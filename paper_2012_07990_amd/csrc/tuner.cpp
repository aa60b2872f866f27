// Autotuner (Auto-tuning subsection of the Compiler Implementation section):
// the valid schedules of an algorithm -- load balancing x direction /
// hybrid threshold x frontier representation and creation x deduplication x
// kernel fusion x delta x EdgeBlocking width -- are timed on the graph and
// narrowed by successive halving (every round keeps the faster half and
// doubles the number of probe sources each survivor is timed on) within a
// wall-clock budget.
// The winner is cached on the graph per algorithm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "algos.hpp"

namespace gg {

static gg_simple_schedule base_simple() { return default_schedule().s1; }

static std::vector<gg_schedule> candidates(const Graph &G, int algo) {
    std::vector<gg_schedule> out;
    auto push = [&](const gg_schedule &s) {
        try {
            validate_schedule(G, algo, s);
            out.push_back(s);
        } catch (const Error &) {
        }
    };
    const int lbs[] = {GG_LB_VERTEX_BASED, GG_LB_WM, GG_LB_CM, GG_LB_STRICT, GG_LB_TWC, GG_LB_ETWC, GG_LB_EDGE_ONLY};
    const float thetas[] = {0.001f, 0.01f, 0.05f, 0.2f};
    // output-frontier creation x deduplication of a push step (configFrontierCreation,
    // configDeduplication): FUSED with each dedup kind or none, and the two dense
    // forms (duplicate-free by construction)
    struct CreateDedup {
        int create, dedup_on, dedup;
    };
    const CreateDedup cds[] = {{GG_CREATE_FUSED, 1, GG_DEDUP_MONOTONIC_COUNTERS},
                               {GG_CREATE_FUSED, 1, GG_DEDUP_BITMAP},
                               {GG_CREATE_FUSED, 1, GG_DEDUP_BOOLMAP},
                               {GG_CREATE_FUSED, 0, GG_DEDUP_MONOTONIC_COUNTERS},
                               {GG_CREATE_UNFUSED_BOOLMAP, 0, GG_DEDUP_MONOTONIC_COUNTERS},
                               {GG_CREATE_UNFUSED_BITMAP, 0, GG_DEDUP_MONOTONIC_COUNTERS}};
    auto with_cd = [](gg_simple_schedule x, const CreateDedup &cd) {
        x.frontier_creation = cd.create;
        x.dedup_enable = cd.dedup_on;
        x.dedup_type = cd.dedup;
        return x;
    };
    gg_schedule s = default_schedule();
    switch (algo) {
    case GG_ALGO_BFS:
    case GG_ALGO_BC:
        for (int lb : lbs) {
            s = default_schedule();
            s.s1.load_balance = lb;
            // push only, under every creation x dedup choice (BC keeps its
            // levels as queues: only the dedup choices differ there)
            for (const CreateDedup &cd : cds) {
                if (algo == GG_ALGO_BC && cd.create != GG_CREATE_FUSED) continue;
                gg_schedule p = s;
                p.s1 = with_cd(s.s1, cd);
                push(p);
            }
            for (float th : thetas)
                for (int rep : {GG_REP_BITMAP, GG_REP_BOOLMAP}) {
                    gg_schedule h = s;
                    h.hybrid = 1;
                    h.threshold = th;
                    h.s2 = base_simple();
                    h.s2.direction = GG_PULL;
                    h.s2.pull_rep = rep;
                    h.s2.dedup_enable = 0;
                    h.s2.frontier_creation = algo == GG_ALGO_BFS ? GG_CREATE_UNFUSED_BITMAP : GG_CREATE_FUSED;
                    push(h);
                }
            if (algo == GG_ALGO_BFS) {
                gg_schedule f = s;
                f.s1.kernel_fusion = 1;
                push(f);
                gg_schedule fh = f;
                fh.hybrid = 1;
                fh.threshold = 0.01f;
                fh.s2 = f.s1;
                fh.s2.kernel_fusion = 0;
                fh.s2.direction = GG_PULL;
                fh.s2.pull_rep = GG_REP_BITMAP;
                push(fh);
            }
        }
        break;
    case GG_ALGO_SSSP:
        // the near queue stays a queue: SSSP varies the deduplication only.
        // Wide buckets first: the first halving round times every candidate
        // once in this order, and a budget that runs out there keeps the
        // narrow-bucket ones (the slowest on every graph measured) untimed
        for (int delta : {4096, 512, 64, 8, 1}) {
            for (int lb : lbs)
                for (int fused : {0, 1})
                    for (const CreateDedup &cd : cds) {
                        if (cd.create != GG_CREATE_FUSED) continue;
                        if (fused && !(cd.dedup_on && cd.dedup == GG_DEDUP_MONOTONIC_COUNTERS)) continue;
                        s = default_schedule();
                        s.s1 = with_cd(s.s1, cd);
                        s.s1.load_balance = lb;
                        s.s1.delta = delta;
                        s.s1.kernel_fusion = fused;
                        push(s);
                    }
            // sparse rounds with STRICT, dense rounds over the EdgeBlocked COO
            // (next to the same bucket width's single schedules)
            if (delta < 512) continue;
            for (int lg : {20, 21})
                for (float th : {0.1f, 0.2f}) {
                    if ((1 << lg) >= G.n) continue;
                    s = default_schedule();
                    s.s1.load_balance = GG_LB_STRICT;
                    s.s1.delta = delta;
                    s.hybrid = 1;
                    s.threshold = th;
                    s.s2 = s.s1;
                    s.s2.load_balance = GG_LB_EDGE_ONLY;
                    s.s2.edge_blocking = 1;
                    s.s2.blocking_size = 1 << lg;
                    s.s2.frontier_creation = GG_CREATE_UNFUSED_BOOLMAP;
                    push(s);
                }
        }
        break;
    case GG_ALGO_CC:
        for (int lb : lbs)
            for (int fused : {0, 1}) {
                s = default_schedule();
                s.s1.load_balance = lb;
                s.s1.kernel_fusion = fused;
                push(s);
            }
        // the hook sweep over pairs blocked by destination segment
        for (int lg = 17; lg <= 22; lg++) {
            if ((1 << lg) >= G.n || ((long long)G.n + (1 << lg) - 1) >> lg > 64) continue;
            s = default_schedule();
            s.s1.load_balance = GG_LB_EDGE_ONLY;
            s.s1.edge_blocking = 1;
            s.s1.blocking_size = 1 << lg;
            push(s);
        }
        break;
    case GG_ALGO_PR:
        for (int lb : {GG_LB_VERTEX_BASED, GG_LB_WM, GG_LB_ETWC, GG_LB_STRICT}) {
            s = default_schedule();
            s.s1.direction = GG_PULL;
            s.s1.load_balance = lb;
            push(s);
        }
        s = default_schedule();
        s.s1.load_balance = GG_LB_EDGE_ONLY;
        push(s);
        for (int lg = 17; lg <= 22; lg++) {
            if ((1 << lg) >= G.n) break;
            s = default_schedule();
            s.s1.direction = GG_PULL;
            s.s1.load_balance = GG_LB_STRICT;
            s.s1.edge_blocking = 1;
            s.s1.blocking_size = 1 << lg;
            push(s);
            s.s1.direction = GG_PUSH;
            s.s1.load_balance = GG_LB_EDGE_ONLY;
            push(s);
        }
        break;
    default:
        throw Error(GG_ERR_INVALID_ARG, "unknown algorithm");
    }
    return out;
}

// One timed run (seconds); the drivers synchronise before returning.
static double time_one(Graph &G, int algo, const gg_schedule &s, int src, void *out1, void *out2, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    switch (algo) {
    case GG_ALGO_BFS: bfs_run(G, src, s, (int32_t *)out1, st, nullptr); break;
    case GG_ALGO_SSSP: sssp_run(G, src, s, (int32_t *)out1, st, nullptr); break;
    case GG_ALGO_CC: cc_run(G, s, (int32_t *)out1, st, nullptr); break;
    case GG_ALGO_PR: pr_run(G, s, 0.85f, 20, 0, (float *)out1, st, nullptr); break;
    case GG_ALGO_BC: bc_run(G, src, s, (uint64_t *)out1, (float *)out2, st, nullptr); break;
    }
    GG_HIP(hipStreamSynchronize(st));
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

gg_schedule autotune(Graph &G, int algo, double budget_s, const int32_t *probes, int nprobe, hipStream_t st,
                     double *best_ms) {
    {
        std::lock_guard<std::mutex> lk(G.mu);
        auto it = G.tuned.find(algo);
        if (it != G.tuned.end() && budget_s <= 0) {
            if (best_ms) *best_ms = it->second.second;
            return it->second.first;
        }
    }
    if (algo == GG_ALGO_SSSP) require(G.has_weights, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
    std::vector<int> srcs;
    for (int i = 0; i < nprobe; i++) {
        require(probes[i] >= 0 && probes[i] < G.n, GG_ERR_INVALID_ARG, "probe source out of range");
        srcs.push_back(probes[i]);
    }
    if (srcs.empty()) srcs.push_back(0);
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    DevBuf<int64_t> o1, o2;
    o1.ensure((size_t)G.n);
    o2.ensure((size_t)G.n);
    struct Cand {
        gg_schedule s;
        double t;
    };
    std::vector<Cand> cands;
    for (auto &s : candidates(G, algo)) cands.push_back({s, 1e30});
    require(!cands.empty(), GG_ERR_UNSUPPORTED_SCHEDULE, "no valid schedule to tune");
    // the EdgeBlocked layouts the candidates read are preprocessing, built
    // once per graph and width before any candidate is timed
    {
        Ctx c;
        c.s = st;
        c.num_cus = G.num_cus;
        for (const Cand &cd : cands)
            for (const gg_simple_schedule *x : {&cd.s.s1, &cd.s.s2}) {
                if (x == &cd.s.s2 && !cd.s.hybrid) continue;
                if (!x->edge_blocking) continue;
                if (algo == GG_ALGO_SSSP) edgeblock_prepare(c, G, x->blocking_size);
                else if (algo == GG_ALGO_PR && x->direction == GG_PULL) pull_layout_prepare(G, x->blocking_size, st);
            }
    }
    t0 = std::chrono::steady_clock::now();  // the search budget starts here
    // A candidate's time in a round is the sum over that round's sources (the
    // same sources for every candidate), so a schedule that is slow on some
    // sources loses even when it is fast on others; the first round runs each
    // candidate once untimed first (a workspace grown on first use).
    int runs = 1, probe_i = 0;
    bool first = true;
    while (cands.size() > 1) {
        size_t timed = 0;
        for (auto &c : cands) {
            double sum = 0;
            try {
                if (first) time_one(G, algo, c.s, srcs[0], o1.p, o2.p, st);
                for (int r = 0; r < runs; r++) {
                    const int src = srcs[(probe_i + r) % srcs.size()];
                    sum += time_one(G, algo, c.s, src, o1.p, o2.p, st);
                }
            } catch (const Error &e) {
                if (e.code == GG_ERR_DEVICE) throw;
                sum = 1e30;  // e.g. a queue overflow without dedup: not a usable schedule
            }
            c.t = sum / runs;
            timed++;
            if (elapsed() > budget_s) break;
        }
        // a round cut short by the budget: only the candidates it timed (the
        // front of the previous ranking) compete, on the same sources
        if (timed < cands.size()) cands.resize(timed);
        std::stable_sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.t < b.t; });
        if (elapsed() > budget_s) break;
        cands.resize((cands.size() + 1) / 2);
        probe_i += runs;
        runs *= 2;
        first = false;
    }
    const Cand &w = cands.front();
    if (best_ms) *best_ms = w.t * 1e3;
    std::lock_guard<std::mutex> lk(G.mu);
    G.tuned[algo] = {w.s, w.t * 1e3};
    return w.s;
}

}  // namespace gg
