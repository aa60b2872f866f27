// Serving loop on the GPU: a serve::Core (admission + continuous batching)
// driven by an executor that runs batches on its own HIP streams. BFS and
// SSSP queries of one graph are batched up to 64, BC queries up to 16; CC
// and PageRank run one query per launch. Batched SSSP is a shared-bucket
// delta-stepping loop; batched BFS is the bit-packed PULL sweep on
// low-diameter graphs and the unit-weight form of the SSSP loop on sparse,
// high-diameter ones, where single queries take the batched loops too (they
// are persistent). Every worker owns a default-priority stream, so batches of
// different graphs and algorithms overlap on the device. A batch that runs a
// persistent (fused) loop takes the device exclusively: its co-resident grid
// assumes no other kernel occupies the compute units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <shared_mutex>

#include "algos.hpp"
#include "handles.hpp"
#include "serve_core.hpp"

namespace gg {

static_assert(serve::kAdmissionStatus == GG_ERR_ADMISSION, "admission status mismatch");

struct GpuExecutor : serve::Executor {
    static constexpr int kMaxGraphs = 64;
    Graph *graphs[kMaxGraphs] = {};
    int ngraphs = 0;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::map<std::pair<int, int>, gg_schedule> sched;
    // a persistent (fused) loop assumes the whole device: it runs alone
    std::shared_mutex device;

    hipStream_t release_stream = nullptr;

    explicit GpuExecutor(int workers) {
        for (int i = 0; i < workers; i++) {
            hipStream_t s;
            GG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            streams.push_back(s);
        }
        GG_HIP(hipStreamCreateWithFlags(&release_stream, hipStreamNonBlocking));
    }
    ~GpuExecutor() override {
        for (auto s : streams) (void)hipStreamSynchronize(s);
        if (release_stream) (void)hipStreamSynchronize(release_stream);
        for (auto s : streams) (void)hipStreamDestroy(s);
        if (release_stream) (void)hipStreamDestroy(release_stream);
    }

    // SSSP on dense (low-diameter) graphs runs one query per launch: the
    // batched delta-stepping loop gains nothing there (measured on R-MAT 20:
    // 2.66 ms per query batched against 2.50 ms single) and, being
    // persistent, would take the device exclusively, while single queries
    // overlap with the other streams' batches
    int max_batch(int gid, int algo) const override {
        if (algo == GG_ALGO_SSSP) return dense(gid) ? 1 : 64;
        return algo == GG_ALGO_BFS ? 64 : algo == GG_ALGO_BC ? 16 : 1;
    }
    bool dense(int gid) const { return graphs[gid]->m >= 8ll * graphs[gid]->n; }

    size_t result_bytes(int gid, int algo) const override {
        const size_t n = (size_t)graphs[gid]->n;
        return algo == GG_ALGO_BC ? 12 * n : 4 * n;
    }
    size_t work_bytes(int gid, int algo, int k) const override {
        // workspace plus the batch output staged before it is split per query
        const size_t stage = k > 1 ? (size_t)k * result_bytes(gid, algo) : 0;
        return workspace_bytes(*graphs[gid], algo, k) + stage;
    }

    gg_schedule schedule_for(int gid, int algo) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = sched.find({gid, algo});
        if (it != sched.end()) return it->second;
        Graph &G = *graphs[gid];
        {
            std::lock_guard<std::mutex> lg(G.mu);
            auto t = G.tuned.find(algo);
            if (t != G.tuned.end() && !t->second.first.s1.kernel_fusion) return t->second.first;
        }
        gg_schedule s = preset_schedule(algo, GG_PRESET_POWERLAW);
        // STRICT push measured fastest on R-MAT for BFS, SSSP and BC
        if (algo == GG_ALGO_BFS || algo == GG_ALGO_SSSP || algo == GG_ALGO_BC) s.s1.load_balance = GG_LB_STRICT;
        // high-diameter graphs: batched BFS as the sparse-queue push loop
        if (algo == GG_ALGO_BFS && G.m < 8ll * G.n) s = default_schedule();
        // wide buckets: fewer rounds (each a grid barrier or a launch) against
        // some re-relaxed edges; measured fastest on both R-MAT and the grids
        if (algo == GG_ALGO_SSSP) s.s1.delta = 4096;
        if (algo == GG_ALGO_SSSP && !G.has_weights) s = default_schedule();
        return s;
    }

    // Stream-ordered device buffer freed on every exit path.
    struct AsyncBuf {
        void *p = nullptr;
        hipStream_t s;
        explicit AsyncBuf(hipStream_t st) : s(st) {}
        AsyncBuf(const AsyncBuf &) = delete;
        ~AsyncBuf() {
            if (p) (void)hipFreeAsync(p, s);
        }
    };

    void fail(serve::Batch &b, hipStream_t st, int code) {
        (void)hipStreamSynchronize(st);
        for (auto *r : b.reqs) {
            r->status = code;
            if (r->result) (void)hipFreeAsync(r->result, st);
            r->result = nullptr;
        }
    }

    void run(int worker, serve::Batch &b) override {
        hipStream_t st = streams[worker];
        Graph &G = *graphs[b.gid];
        const size_t n = (size_t)G.n;
        const int k = (int)b.reqs.size();
        const gg_schedule s = schedule_for(b.gid, b.algo);
        // the batched loops also serve single queries where they are persistent
        // push loops (SSSP always; BFS under a plain PUSH schedule)
        const bool ms_push = b.algo == GG_ALGO_SSSP || (b.algo == GG_ALGO_BFS && !s.hybrid && s.s1.direction == GG_PUSH);
        const bool batched = k > 1 || (ms_push && G.m < 8ll * G.n);
        // persistent: the push loops, and the pull forms under a fused schedule
        const bool fused = (batched && ms_push) || s.s1.kernel_fusion;
        std::shared_lock<std::shared_mutex> shared(device, std::defer_lock);
        std::unique_lock<std::shared_mutex> exclusive(device, std::defer_lock);
        if (fused) exclusive.lock();
        else shared.lock();
        try {
            for (serve::Req *r : b.reqs) GG_HIP(hipMallocAsync(&r->result, r->result_bytes, st));
            if (!batched) {
                serve::Req *r = b.reqs[0];
                switch (b.algo) {
                case GG_ALGO_BFS: bfs_run(G, r->src, s, (int32_t *)r->result, st, nullptr); break;
                case GG_ALGO_SSSP: sssp_run(G, r->src, s, (int32_t *)r->result, st, nullptr); break;
                case GG_ALGO_CC: cc_run(G, s, (int32_t *)r->result, st, nullptr); break;
                case GG_ALGO_PR: pr_run(G, s, 0.85f, 20, 0, (float *)r->result, st, nullptr); break;
                case GG_ALGO_BC:
                    bc_run(G, r->src, s, (uint64_t *)r->result, (float *)((char *)r->result + 8 * n), st, nullptr);
                    break;
                }
                GG_HIP(hipStreamSynchronize(st));
                for (auto *r2 : b.reqs) r2->status = GG_OK;
                return;
            }
            std::vector<int32_t> srcs;
            for (auto *r : b.reqs) srcs.push_back(r->src);
            AsyncBuf stage(st);
            GG_HIP(hipMallocAsync(&stage.p, (size_t)k * result_bytes(b.gid, b.algo), st));
            unsigned long long overflow = 0;
            if (b.algo == GG_ALGO_BFS || b.algo == GG_ALGO_SSSP) {
                if (b.algo == GG_ALGO_BFS) msbfs_run(G, srcs.data(), k, s, (int32_t *)stage.p, st, nullptr);
                else mssssp_run(G, srcs.data(), k, s, (int32_t *)stage.p, st, nullptr, &overflow);
                for (int i = 0; i < k; i++)
                    GG_HIP(hipMemcpyAsync(b.reqs[i]->result, (int32_t *)stage.p + i * n, 4 * n,
                                          hipMemcpyDeviceToDevice, st));
            } else {
                uint64_t *sig = (uint64_t *)stage.p;
                float *del = (float *)((char *)stage.p + 8 * n * k);
                msbc_run(G, srcs.data(), k, s, sig, del, st, nullptr);
                for (int i = 0; i < k; i++) {
                    GG_HIP(hipMemcpyAsync(b.reqs[i]->result, sig + i * n, 8 * n, hipMemcpyDeviceToDevice, st));
                    GG_HIP(hipMemcpyAsync((char *)b.reqs[i]->result + 8 * n, del + i * n, 4 * n,
                                          hipMemcpyDeviceToDevice, st));
                }
            }
            GG_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < k; i++) {
                serve::Req *r = b.reqs[i];
                r->status = ((overflow >> i) & 1ull) ? GG_ERR_OVERFLOW : GG_OK;
                if (r->status != GG_OK) {
                    (void)hipFreeAsync(r->result, st);
                    r->result = nullptr;
                }
            }
        } catch (const Error &e) {
            fail(b, st, e.code);
        } catch (const std::bad_alloc &) {
            fail(b, st, GG_ERR_OUT_OF_MEMORY);
        } catch (const std::exception &) {
            fail(b, st, GG_ERR_DEVICE);
        }
    }

    // results were complete on their worker's stream before the client saw
    // them; they go back to the stream-ordered pool through the release stream
    void release(serve::Req &r) override {
        if (r.result) (void)hipFreeAsync(r.result, release_stream);
        r.result = nullptr;
    }

    // derived layouts a graph already had when it was added belong to the
    // caller's graph (like its CSR); those built since are charged
    size_t layout_base[kMaxGraphs] = {};
    size_t pinned_bytes() override {
        size_t b = 0;
        for (int i = 0; i < ngraphs; i++) {
            const size_t l = graphs[i]->layout_bytes();
            b += l > layout_base[i] ? l - layout_base[i] : 0;
        }
        return b;
    }
    size_t idle_bytes() override {
        size_t b = pinned_bytes();
        for (int i = 0; i < ngraphs; i++) b += graphs[i]->pooled_bytes();
        return b;
    }

    // derived layouts stay; pooled workspaces are freed, largest graphs' first
    void trim(size_t target) override {
        size_t idle = idle_bytes();
        std::vector<int> order;
        for (int i = 0; i < ngraphs; i++) order.push_back(i);
        std::sort(order.begin(), order.end(), [&](int a, int b2) { return graphs[a]->n > graphs[b2]->n; });
        for (int i : order) {
            if (idle <= target) break;
            const size_t pooled = graphs[i]->pooled_bytes();
            const size_t excess = idle - target;
            idle -= graphs[i]->trim_pool(pooled > excess ? pooled - excess : 0);
        }
    }
};

}  // namespace gg

using namespace gg;

struct gg_server {
    std::unique_ptr<GpuExecutor> ex;
    std::unique_ptr<serve::Core> core;
    size_t budget = 0;
};

template <class Fn>
static gg_status sguard(Fn &&fn) {
    try {
        fn();
        g_last_error.clear();
        return GG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const serve::AdmissionError &e) {
        g_last_error = e.what();
        return GG_ERR_ADMISSION;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GG_ERR_DEVICE;
    }
}

static void fill_result(const serve::Req &r, gg_result *res) {
    if (!res) return;
    res->ticket = r.ticket;
    res->status = r.status;
    res->graph_id = r.gid;
    res->algo = r.algo;
    res->src = r.src;
    res->batch_size = r.batch_size;
    res->queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_arrive).count();
    res->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_arrive).count();
}

static gg_status deliver(gg_server *srv, const serve::Req &r, void *out, uint32_t flags, gg_result *res) {
    fill_result(r, res);
    if (r.status == GG_OK && out && !(flags & GG_OUT_DISCARD) && r.result) {
        const hipMemcpyKind k = (flags & GG_OUT_HOST) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (hipMemcpy(out, r.result, r.result_bytes, k) != hipSuccess) return GG_ERR_DEVICE;
    }
    srv->core->collect(r.ticket);
    return GG_OK;
}

extern "C" {

gg_status gg_server_create(size_t hbm_budget, int32_t nstreams, gg_server **out) {
    return sguard([&] {
        require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        require(hbm_budget > 0, GG_ERR_INVALID_ARG, "budget must be > 0");
        require(nstreams >= 1 && nstreams <= 16, GG_ERR_INVALID_ARG, "nstreams must be in [1, 16]");
        auto s = std::make_unique<gg_server>();
        s->ex = std::make_unique<GpuExecutor>(nstreams);
        s->budget = hbm_budget;
        s->core = std::make_unique<serve::Core>(s->ex.get(), hbm_budget, nstreams);
        *out = s.release();
    });
}

gg_status gg_server_add_graph(gg_server *srv, gg_graph *g, int32_t *gid) {
    return sguard([&] {
        require(srv && g && gid, GG_ERR_INVALID_ARG, "NULL argument");
        require(srv->core->stats().submitted == 0, GG_ERR_INVALID_ARG, "add every graph before the first query");
        require(srv->ex->ngraphs < GpuExecutor::kMaxGraphs, GG_ERR_INVALID_ARG, "too many graphs");
        require(g->g.symmetric, GG_ERR_INVALID_ARG, "served graphs must be symmetric (GG_SYMMETRIC)");
        srv->ex->graphs[srv->ex->ngraphs] = &g->g;
        srv->ex->layout_base[srv->ex->ngraphs] = g->g.layout_bytes();
        *gid = srv->ex->ngraphs++;
    });
}

gg_status gg_server_set_schedule(gg_server *srv, int32_t gid, int32_t algo, const gg_schedule *s) {
    return sguard([&] {
        require(srv && s, GG_ERR_INVALID_ARG, "NULL argument");
        require(gid >= 0 && gid < srv->ex->ngraphs, GG_ERR_INVALID_ARG, "unknown graph id");
        validate_schedule(*srv->ex->graphs[gid], algo, *s);
        std::lock_guard<std::mutex> lk(srv->ex->mu);
        srv->ex->sched[{gid, algo}] = *s;
    });
}

gg_status gg_server_submit(gg_server *srv, int32_t gid, int32_t algo, int32_t src, int64_t *ticket) {
    return sguard([&] {
        require(srv && ticket, GG_ERR_INVALID_ARG, "NULL argument");
        require(gid >= 0 && gid < srv->ex->ngraphs, GG_ERR_INVALID_ARG, "unknown graph id");
        require(algo >= GG_ALGO_BFS && algo <= GG_ALGO_BC, GG_ERR_INVALID_ARG, "unknown algorithm");
        const Graph &G = *srv->ex->graphs[gid];
        require(src >= 0 && src < G.n, GG_ERR_INVALID_ARG, "source out of range");
        require(algo != GG_ALGO_SSSP || G.has_weights, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
        *ticket = srv->core->submit(gid, algo, src);
    });
}

gg_status gg_server_poll(gg_server *srv, int64_t ticket, void *out, uint32_t flags, gg_result *res) {
    gg_status st = sguard([&] {
        require(srv != nullptr, GG_ERR_INVALID_ARG, "server is NULL");
        require(srv->core->known(ticket), GG_ERR_NOT_FOUND, "unknown ticket");
    });
    if (st != GG_OK) return st;
    serve::Req r;
    if (!srv->core->peek(ticket, r)) return GG_ERR_NOT_READY;
    st = deliver(srv, r, out, flags, res);
    return st != GG_OK ? st : (gg_status)r.status;
}

gg_status gg_server_wait(gg_server *srv, int64_t ticket, double timeout_s, void *out, uint32_t flags,
                         gg_result *res) {
    gg_status st = sguard([&] {
        require(srv != nullptr, GG_ERR_INVALID_ARG, "server is NULL");
        require(srv->core->known(ticket), GG_ERR_NOT_FOUND, "unknown ticket");
    });
    if (st != GG_OK) return st;
    serve::Req r;
    if (!srv->core->wait(ticket, timeout_s, r)) return GG_ERR_NOT_READY;
    st = deliver(srv, r, out, flags, res);
    return st != GG_OK ? st : (gg_status)r.status;
}

gg_status gg_server_stats(gg_server *srv, gg_serve_stats *out) {
    return sguard([&] {
        require(srv && out, GG_ERR_INVALID_ARG, "NULL argument");
        const serve::Stats s = srv->core->stats();
        out->submitted = s.submitted;
        out->completed = s.completed;
        out->collected = s.collected;
        out->rejected = s.rejected;
        out->batches = s.batches;
        out->max_batch = s.max_batch_seen;
        out->bytes_in_use = s.bytes_in_use;
        out->bytes_peak = s.bytes_peak;
        out->busy_ms = s.busy_ms;
        out->bytes_idle = s.bytes_idle;
        out->trims = s.trims;
    });
}

gg_status gg_server_destroy(gg_server *srv) {
    return sguard([&] {
        if (!srv) return;
        srv->core->shutdown();
        srv->core.reset();
        srv->ex.reset();
        delete srv;
    });
}

}  // extern "C"
