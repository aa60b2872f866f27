// C ABI: argument validation, graph creation, schedule defaults/validation
// and dispatch to the algorithm drivers. No C++ exception crosses this file's
// extern "C" functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "algos.hpp"
#include "handles.hpp"
#include "ops.hpp"

using namespace gg;

namespace gg {
thread_local std::string g_last_error;
}

template <class Fn>
static gg_status guarded(Fn &&fn) {
    try {
        fn();
        g_last_error.clear();
        return GG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GG_ERR_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GG_ERR_DEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return GG_ERR_DEVICE;
    }
}

namespace gg {

std::unique_ptr<Workspace> Graph::acquire() {
    std::unique_ptr<Workspace> w;
    std::lock_guard<std::mutex> lk(mu);
    if (!pool.empty()) {
        w = std::move(pool.back());
        pool.pop_back();
    } else {
        w = std::make_unique<Workspace>();
    }
    w->lease_bytes = w->bytes();
    leased += w->lease_bytes;
    return w;
}

void Graph::give_back(std::unique_ptr<Workspace> ws) {
    if (!ws) return;
    std::unique_ptr<Workspace> drop;
    {
        std::lock_guard<std::mutex> lk(mu);
        leased -= ws->lease_bytes;
        ws->lease_bytes = 0;
        if (pool.size() < 8) pool.push_back(std::move(ws));
        else drop = std::move(ws);
    }
}

size_t Graph::pooled_bytes() {
    std::lock_guard<std::mutex> lk(mu);
    size_t b = leased;
    for (auto &w : pool) b += w->bytes();
    return b;
}

size_t Graph::layout_bytes() {
    std::lock_guard<std::mutex> lk(mu);
    size_t b = coo_src.bytes() + upper.bytes() + in_rp.bytes() + in_col.bytes();
    for (auto &kv : eb) b += kv.second->src.bytes() + kv.second->dst.bytes() + kv.second->w.bytes();
    for (auto &kv : upper_eb) b += kv.second->pairs.bytes();
    for (auto &kv : pull_eb) {
        const PullBlocked &p = *kv.second;
        b += p.rp.bytes() + p.col.bytes() + p.chunk_rows.bytes() + p.hot_slot.bytes() + p.hcol.bytes();
    }
    return b;
}

size_t Graph::trim_pool(size_t keep) {
    std::vector<std::unique_ptr<Workspace>> drop;
    size_t freed = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        size_t held = leased;
        for (auto &w : pool) held += w->bytes();
        while (!pool.empty() && held > keep) {
            const size_t b = pool.back()->bytes();
            held -= b;
            freed += b;
            drop.push_back(std::move(pool.back()));
            pool.pop_back();
        }
    }
    drop.clear();  // the buffers are freed outside the lock
    return freed;
}

}  // namespace gg

static hipStream_t S(gg_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

static void check_graph(const gg_graph *g) { require(g != nullptr, GG_ERR_INVALID_ARG, "graph is NULL"); }

static void validate_csr_host(int32_t n, int64_t m, const int32_t *rp, const int32_t *col) {
    require(rp[0] == 0, GG_ERR_INVALID_ARG, "row_ptr[0] != 0");
    require(rp[n] == m, GG_ERR_INVALID_ARG, "row_ptr[n] != m");
    for (int32_t v = 0; v < n; v++) {
        require(rp[v + 1] >= rp[v], GG_ERR_INVALID_ARG, "row_ptr not monotone at " + std::to_string(v));
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            require(col[e] >= 0 && col[e] < n, GG_ERR_INVALID_ARG, "col out of range at entry " + std::to_string(e));
            require(col[e] != v, GG_ERR_INVALID_ARG, "self-loop at vertex " + std::to_string(v));
            require(e == rp[v] || col[e] > col[e - 1], GG_ERR_INVALID_ARG,
                    "row " + std::to_string(v) + " not strictly ascending");
        }
    }
}

extern "C" {

const char *gg_status_string(gg_status s) {
    switch (s) {
    case GG_OK: return "ok";
    case GG_ERR_INVALID_ARG: return "invalid argument";
    case GG_ERR_OUT_OF_MEMORY: return "out of memory";
    case GG_ERR_DEVICE: return "device error";
    case GG_ERR_UNSUPPORTED_SCHEDULE: return "unsupported schedule";
    case GG_ERR_OVERFLOW: return "overflow";
    case GG_ERR_ADMISSION: return "admission refused";
    case GG_ERR_NOT_FOUND: return "not found";
    case GG_ERR_NOT_READY: return "not ready";
    }
    return "unknown status";
}

const char *gg_last_error(void) { return g_last_error.c_str(); }

const char *gg_version(void) { return "gg-mi355x 0.1 (gfx950)"; }

gg_status gg_graph_create_csr(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                              uint32_t flags, gg_stream_t stream, gg_graph **out) {
    return guarded([&] {
        require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        require(n >= 1, GG_ERR_INVALID_ARG, "n must be >= 1");
        require(m >= 0 && m < (int64_t(1) << 31), GG_ERR_INVALID_ARG, "m must be in [0, 2^31)");
        require(row_ptr != nullptr, GG_ERR_INVALID_ARG, "row_ptr is NULL");
        require(m == 0 || col != nullptr, GG_ERR_INVALID_ARG, "col is NULL");
        const bool dev = flags & GG_INPUT_DEVICE;
        hipStream_t s = S(stream);
        auto G = std::make_unique<gg_graph>();
        Graph &g = G->g;
        g.n = n;
        g.m = m;
        g.symmetric = flags & GG_SYMMETRIC;
        g.has_weights = w != nullptr;
        GG_HIP(hipGetDevice(&g.device));
        GG_HIP(hipDeviceGetAttribute(&g.num_cus, hipDeviceAttributeMultiprocessorCount, g.device));
        // host copies for validation / statistics
        std::vector<int32_t> hrp((size_t)n + 1);
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
        GG_HIP(hipMemcpy(hrp.data(), row_ptr, sizeof(int32_t) * (n + 1), kind));
        require(hrp[0] == 0 && hrp[n] == m, GG_ERR_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n] must be m");
        if (flags & GG_VALIDATE) {
            std::vector<int32_t> hcol((size_t)m);
            if (m) GG_HIP(hipMemcpy(hcol.data(), col, sizeof(int32_t) * m, kind));
            validate_csr_host(n, m, hrp.data(), hcol.data());
            if (w) {
                std::vector<uint32_t> hw((size_t)m);
                if (m) GG_HIP(hipMemcpy(hw.data(), w, sizeof(uint32_t) * m, kind));
                for (int64_t e = 0; e < m; e++)
                    require(hw[e] >= 1, GG_ERR_INVALID_ARG, "edge weights must be >= 1");
            }
        }
        int32_t maxd = 0;
        for (int32_t v = 0; v < n; v++) maxd = std::max(maxd, hrp[v + 1] - hrp[v]);
        g.max_degree = maxd;
        g.row_ptr.ensure((size_t)n + 1);
        g.col.ensure((size_t)std::max<int64_t>(m, 1));
        const hipMemcpyKind k2 = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        GG_HIP(hipMemcpyAsync(g.row_ptr.p, hrp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
        if (m) GG_HIP(hipMemcpyAsync(g.col.p, col, sizeof(int32_t) * m, k2, s));
        if (w) {
            g.w.ensure((size_t)std::max<int64_t>(m, 1));
            if (m) GG_HIP(hipMemcpyAsync(g.w.p, w, sizeof(uint32_t) * m, k2, s));
        }
        GG_HIP(hipStreamSynchronize(s));
        *out = G.release();
    });
}

gg_status gg_graph_destroy(gg_graph *g) {
    return guarded([&] { delete g; });
}

gg_status gg_graph_info(const gg_graph *g, int32_t *n, int64_t *m, int32_t *has_weights, int32_t *symmetric) {
    return guarded([&] {
        check_graph(g);
        if (n) *n = g->g.n;
        if (m) *m = g->g.m;
        if (has_weights) *has_weights = g->g.has_weights;
        if (symmetric) *symmetric = g->g.symmetric;
    });
}

gg_status gg_graph_prepare_edgeblocking(gg_graph *g, int32_t seg_vertices, gg_stream_t stream, double *prep_ms) {
    return guarded([&] {
        check_graph(g);
        require(seg_vertices >= 1, GG_ERR_INVALID_ARG, "seg_vertices must be >= 1");
        Ctx c;
        c.s = S(stream);
        c.num_cus = g->g.num_cus;
        double ms = edgeblock_prepare(c, g->g, seg_vertices);
        if (prep_ms) *prep_ms = ms;
    });
}

gg_status gg_graph_prepare_pull_blocking(gg_graph *g, int32_t seg_vertices, gg_stream_t stream, double *prep_ms) {
    return guarded([&] {
        check_graph(g);
        require(seg_vertices >= 1, GG_ERR_INVALID_ARG, "seg_vertices must be >= 1");
        const double ms = pull_layout_prepare(g->g, seg_vertices, S(stream));
        if (prep_ms) *prep_ms = ms;
    });
}

gg_status gg_graph_edgeblocking_export(const gg_graph *g, int32_t seg_vertices, int32_t *src_dev, int32_t *dst_dev,
                                       int64_t *seg_start_host, gg_stream_t stream) {
    return guarded([&] {
        check_graph(g);
        Graph &G = const_cast<gg_graph *>(g)->g;
        std::lock_guard<std::mutex> lk(G.mu);
        auto it = G.eb.find(seg_vertices);
        require(it != G.eb.end(), GG_ERR_INVALID_ARG, "EdgeBlocking with this segment size was not prepared");
        const EdgeBlocked &b = *it->second;
        hipStream_t s = S(stream);
        if (G.m) {
            require(src_dev && dst_dev, GG_ERR_INVALID_ARG, "NULL output");
            GG_HIP(hipMemcpyAsync(src_dev, b.src.p, sizeof(int32_t) * G.m, hipMemcpyDeviceToDevice, s));
            GG_HIP(hipMemcpyAsync(dst_dev, b.dst.p, sizeof(int32_t) * G.m, hipMemcpyDeviceToDevice, s));
        }
        if (seg_start_host)
            for (size_t i = 0; i < b.seg_start.size(); i++) seg_start_host[i] = b.seg_start[i];
        GG_HIP(hipStreamSynchronize(s));
    });
}

gg_status gg_schedule_default(gg_schedule *s) {
    return guarded([&] {
        require(s != nullptr, GG_ERR_INVALID_ARG, "schedule is NULL");
        *s = default_schedule();
    });
}

gg_status gg_schedule_preset(int32_t algo, int32_t preset, gg_schedule *s) {
    return guarded([&] {
        require(s != nullptr, GG_ERR_INVALID_ARG, "schedule is NULL");
        *s = preset_schedule(algo, preset);
    });
}

gg_status gg_schedule_validate(const gg_graph *g, int32_t algo, const gg_schedule *s) {
    return guarded([&] {
        check_graph(g);
        require(s != nullptr, GG_ERR_INVALID_ARG, "schedule is NULL");
        validate_schedule(g->g, algo, *s);
    });
}

gg_status gg_bfs(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *depth_dev, gg_stream_t stream,
                 gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(src >= 0 && src < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(depth_dev != nullptr, GG_ERR_INVALID_ARG, "depth is NULL");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(g->g, GG_ALGO_BFS, sc);
        bfs_run(g->g, src, sc, depth_dev, S(stream), stats);
    });
}

gg_status gg_sssp(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *dist_dev, gg_stream_t stream,
                  gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(src >= 0 && src < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(dist_dev != nullptr, GG_ERR_INVALID_ARG, "dist is NULL");
        require(g->g.has_weights, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(g->g, GG_ALGO_SSSP, sc);
        sssp_run(g->g, src, sc, dist_dev, S(stream), stats);
    });
}

gg_status gg_cc(gg_graph *g, const gg_schedule *s, int32_t *label_dev, gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(label_dev != nullptr, GG_ERR_INVALID_ARG, "label is NULL");
        require(g->g.symmetric, GG_ERR_INVALID_ARG, "CC needs a symmetric graph (GG_SYMMETRIC)");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(g->g, GG_ALGO_CC, sc);
        cc_run(g->g, sc, label_dev, S(stream), stats);
    });
}

gg_status gg_pagerank(gg_graph *g, const gg_schedule *s, float damping, int32_t iters, uint32_t flags,
                      float *rank_dev, gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(rank_dev != nullptr, GG_ERR_INVALID_ARG, "rank is NULL");
        require(iters >= 0, GG_ERR_INVALID_ARG, "iters must be >= 0");
        require((flags & ~(GG_PR_NO_DANGLING | GG_PR_NO_LDS_CACHE)) == 0, GG_ERR_INVALID_ARG,
                "unknown PageRank flags");
        require(damping >= 0.f && damping <= 1.f, GG_ERR_INVALID_ARG, "damping must be in [0, 1]");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(g->g, GG_ALGO_PR, sc);
        pr_run(g->g, sc, damping, iters, flags, rank_dev, S(stream), stats);
    });
}

gg_status gg_bc(gg_graph *g, int32_t src, const gg_schedule *s, uint64_t *sigma_dev, float *delta_dev,
                gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(src >= 0 && src < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(sigma_dev && delta_dev, GG_ERR_INVALID_ARG, "sigma/delta is NULL");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(g->g, GG_ALGO_BC, sc);
        bc_run(g->g, src, sc, sigma_dev, delta_dev, S(stream), stats);
    });
}

gg_status gg_bfs_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s, int32_t *depth_dev,
                       gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(k >= 0 && k <= 64, GG_ERR_INVALID_ARG, "k must be in [0, 64]");
        require(k == 0 || (srcs_host && depth_dev), GG_ERR_INVALID_ARG, "NULL sources or output");
        for (int i = 0; i < k; i++)
            require(srcs_host[i] >= 0 && srcs_host[i] < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(g->g.symmetric, GG_ERR_INVALID_ARG, "multi-source BFS needs a symmetric graph (GG_SYMMETRIC)");
        const gg_schedule sc = s ? *s : default_schedule();
        msbfs_run(g->g, srcs_host, k, sc, depth_dev, S(stream), stats);
    });
}

gg_status gg_sssp_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s, int32_t *dist_dev,
                        gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(k >= 0 && k <= 64, GG_ERR_INVALID_ARG, "k must be in [0, 64]");
        require(k == 0 || (srcs_host && dist_dev), GG_ERR_INVALID_ARG, "NULL sources or output");
        for (int i = 0; i < k; i++)
            require(srcs_host[i] >= 0 && srcs_host[i] < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(g->g.has_weights, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
        const gg_schedule sc = s ? *s : default_schedule();
        mssssp_run(g->g, srcs_host, k, sc, dist_dev, S(stream), stats, nullptr);
    });
}

gg_status gg_bc_multi(gg_graph *g, const int32_t *srcs_host, int32_t k, const gg_schedule *s, uint64_t *sigma_dev,
                      float *delta_dev, gg_stream_t stream, gg_stats *stats) {
    return guarded([&] {
        check_graph(g);
        require(k >= 0 && k <= 64, GG_ERR_INVALID_ARG, "k must be in [0, 64]");
        require(k == 0 || (srcs_host && sigma_dev && delta_dev), GG_ERR_INVALID_ARG, "NULL sources or output");
        for (int i = 0; i < k; i++)
            require(srcs_host[i] >= 0 && srcs_host[i] < g->g.n, GG_ERR_INVALID_ARG, "source out of range");
        require(g->g.symmetric, GG_ERR_INVALID_ARG, "multi-source BC needs a symmetric graph (GG_SYMMETRIC)");
        const gg_schedule sc = s ? *s : default_schedule();
        msbc_run(g->g, srcs_host, k, sc, sigma_dev, delta_dev, S(stream), stats);
    });
}

gg_status gg_autotune(gg_graph *g, int32_t algo, double budget_s, const int32_t *probe_srcs, int32_t nprobe,
                      gg_stream_t stream, gg_schedule *out, double *best_ms) {
    return guarded([&] {
        check_graph(g);
        require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        require(algo >= GG_ALGO_BFS && algo <= GG_ALGO_BC, GG_ERR_INVALID_ARG, "unknown algorithm");
        require(nprobe >= 0 && (nprobe == 0 || probe_srcs), GG_ERR_INVALID_ARG, "bad probe sources");
        if (algo == GG_ALGO_CC)
            require(g->g.symmetric, GG_ERR_INVALID_ARG, "CC needs a symmetric graph (GG_SYMMETRIC)");
        *out = autotune(g->g, algo, budget_s, probe_srcs, nprobe, S(stream), best_ms);
    });
}

gg_status gg_tuned_set(gg_graph *g, int32_t algo, const gg_schedule *s, double ms) {
    return guarded([&] {
        check_graph(g);
        require(s != nullptr, GG_ERR_INVALID_ARG, "schedule is NULL");
        require(algo >= GG_ALGO_BFS && algo <= GG_ALGO_BC, GG_ERR_INVALID_ARG, "unknown algorithm");
        validate_schedule(g->g, algo, *s);
        std::lock_guard<std::mutex> lk(g->g.mu);
        g->g.tuned[algo] = {*s, ms};
    });
}

gg_status gg_tuned_get(gg_graph *g, int32_t algo, gg_schedule *out, double *ms) {
    return guarded([&] {
        check_graph(g);
        require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        require(algo >= GG_ALGO_BFS && algo <= GG_ALGO_BC, GG_ERR_INVALID_ARG, "unknown algorithm");
        std::lock_guard<std::mutex> lk(g->g.mu);
        auto it = g->g.tuned.find(algo);
        require(it != g->g.tuned.end(), GG_ERR_NOT_FOUND, "no tuned schedule cached for this algorithm");
        *out = it->second.first;
        if (ms) *ms = it->second.second;
    });
}

gg_status gg_workspace_bytes(const gg_graph *g, int32_t algo, int32_t k, size_t *out) {
    return guarded([&] {
        check_graph(g);
        require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        *out = workspace_bytes(g->g, algo, k);
    });
}

}  // extern "C"
