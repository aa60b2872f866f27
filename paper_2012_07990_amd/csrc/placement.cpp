// CPU-or-GPU placement of one algorithm on one graph (the paper's comparison
// of its CPU and GPU backends on the same algorithm: which target wins
// depends on the graph; delta-stepping on road graphs ran faster on the CPU).
// The decision is measured, not guessed: one warm-up and one timed run of
// the query on each backend, the faster wins, and the result is cached on
// the device graph per algorithm.
#include <hip/hip_runtime.h>

#include <chrono>
#include <vector>

#include "algos.hpp"
#include "handles.hpp"

extern "C" {
gg_status gg_cpu_bfs(gg_cpu_graph *cg, int32_t src, int32_t nthreads, int32_t *depth);
gg_status gg_cpu_sssp(gg_cpu_graph *cg, int32_t src, int32_t delta, int32_t nthreads, int32_t *dist);
gg_status gg_cpu_cc(gg_cpu_graph *cg, int32_t nthreads, int32_t *label);
gg_status gg_cpu_pagerank(gg_cpu_graph *cg, float damping, int32_t iters, uint32_t flags, int32_t nthreads,
                          float *rank);
gg_status gg_cpu_bc(gg_cpu_graph *cg, int32_t src, int32_t nthreads, uint64_t *sigma, float *delta);
}

using namespace gg;

namespace {

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" gg_status gg_place(gg_graph *g, gg_cpu_graph *cg, int32_t algo, const gg_schedule *s, int32_t src,
                              int32_t nthreads, gg_stream_t stream, int32_t *target, double *gpu_ms,
                              double *cpu_ms) {
    try {
        require(g != nullptr && cg != nullptr && target != nullptr, GG_ERR_INVALID_ARG, "NULL argument");
        require(algo >= GG_ALGO_BFS && algo <= GG_ALGO_BC, GG_ERR_INVALID_ARG, "unknown algorithm");
        Graph &G = g->g;
        require(src >= 0 && src < G.n, GG_ERR_INVALID_ARG, "source out of range");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(G, algo, sc);
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        const size_t n = (size_t)G.n;
        DevBuf<unsigned char> dout;
        dout.ensure(12 * n);
        std::vector<unsigned char> hout(12 * n);
        auto gpu_once = [&] {
            switch (algo) {
            case GG_ALGO_BFS: bfs_run(G, src, sc, (int32_t *)dout.p, st, nullptr); break;
            case GG_ALGO_SSSP: sssp_run(G, src, sc, (int32_t *)dout.p, st, nullptr); break;
            case GG_ALGO_CC: cc_run(G, sc, (int32_t *)dout.p, st, nullptr); break;
            case GG_ALGO_PR: pr_run(G, sc, 0.85f, 20, 0, (float *)dout.p, st, nullptr); break;
            default: bc_run(G, src, sc, (uint64_t *)dout.p, (float *)(dout.p + 8 * n), st, nullptr); break;
            }
            GG_HIP(hipStreamSynchronize(st));
        };
        auto cpu_once = [&] {
            gg_status r = GG_OK;
            switch (algo) {
            case GG_ALGO_BFS: r = gg_cpu_bfs(cg, src, nthreads, (int32_t *)hout.data()); break;
            case GG_ALGO_SSSP:
                r = gg_cpu_sssp(cg, src, sc.s1.delta, nthreads, (int32_t *)hout.data());
                break;
            case GG_ALGO_CC: r = gg_cpu_cc(cg, nthreads, (int32_t *)hout.data()); break;
            case GG_ALGO_PR: r = gg_cpu_pagerank(cg, 0.85f, 20, 0, nthreads, (float *)hout.data()); break;
            default:
                r = gg_cpu_bc(cg, src, nthreads, (uint64_t *)hout.data(), (float *)(hout.data() + 8 * n));
                break;
            }
            require(r == GG_OK, r, "CPU backend: " + g_last_error);
        };
        gpu_once();
        auto t0 = std::chrono::steady_clock::now();
        gpu_once();
        const double tg = ms_since(t0);
        cpu_once();
        t0 = std::chrono::steady_clock::now();
        cpu_once();
        const double tc = ms_since(t0);
        *target = tc < tg ? GG_TARGET_CPU : GG_TARGET_GPU;
        if (gpu_ms) *gpu_ms = tg;
        if (cpu_ms) *cpu_ms = tc;
        {
            std::lock_guard<std::mutex> lk(G.mu);
            G.placement[algo] = *target;
        }
        g_last_error.clear();
        return GG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GG_ERR_DEVICE;
    }
}

extern "C" gg_status gg_placement_get(const gg_graph *g, int32_t algo, int32_t *target) {
    try {
        require(g != nullptr && target != nullptr, GG_ERR_INVALID_ARG, "NULL argument");
        const Graph &G = g->g;
        std::lock_guard<std::mutex> lk(const_cast<Graph &>(G).mu);
        auto it = G.placement.find(algo);
        if (it == G.placement.end()) {
            g_last_error = "no placement measured for this algorithm";
            return GG_ERR_NOT_FOUND;
        }
        *target = it->second;
        g_last_error.clear();
        return GG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    }
}
