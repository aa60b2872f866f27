// CPU backend: the five algorithms on a host CSR with a pool of threads, the
// counterpart of the paper's CPU code generation (its Evaluation compares the
// CPU and GPU backends on the same algorithm specification; delta-stepping on
// road graphs ran faster on the CPU). Plain C++17 threads, no device code.
//
// Depths, distances, labels and path counts are unique fixpoints, equal to
// the GPU backend's bit for bit. PageRank and BC dependencies sum each
// vertex's terms in CSR order in fp64 (one thread per vertex) and reduce the
// dangling mass over a fixed chunking, so no result depends on the thread
// count; they match the GPU's within its FP32 tolerances.
//
//   BFS   level-synchronous, direction-optimising: top-down over the frontier
//         (claim a vertex with a compare-and-swap of its depth) while the
//         frontier is small, bottom-up over the unvisited vertices (first
//         parent in the frontier; the transpose on a directed graph) while it
//         holds more than n/20 vertices
//   SSSP  delta-stepping: bucket k = [k delta, (k+1) delta); the current
//         bucket's vertices relax their edges in parallel with an atomic
//         minimum, improved vertices join the current bucket's next round
//         or a later bucket; buckets are visited in increasing order
//   CC    hooking the larger label to the smaller with an atomic minimum,
//         then pointer jumping, until no hook changes anything
//   PR    PULL: rank'(v) = (1-d)/n + d (sum over in-neighbours u of
//         rank(u)/outdeg(u) + D/n), D = rank on vertices without out-edges
//   BC    Brandes: a PULL sweep per level for the path counts (sigma(v) =
//         sum of sigma over parents one level up), then the dependencies
//         level by level from the deepest (delta(v) = sum over successors w
//         of sigma(v)/sigma(w) (1 + delta(w)))
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "handles.hpp"

namespace gg {
namespace cpu {

struct Error {
    gg_status code;
    std::string msg;
};

static void require(bool ok, gg_status code, const std::string &msg) {
    if (!ok) throw Error{code, msg};
}

// ---- a fixed pool of worker threads running parallel-for ranges ----------------------
class Pool {
public:
    explicit Pool(int threads) : nt_(std::max(1, threads)) {
        for (int i = 1; i < nt_; i++) th_.emplace_back([this, i] { loop(i); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    int size() const { return nt_; }
    // f(thread, begin, end) over [0, n) in dynamic chunks of `grain`
    void run(long long n, long long grain, const std::function<void(int, long long, long long)> &f) {
        if (n <= 0) return;
        if (nt_ == 1 || n <= grain) {
            f(0, 0, n);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &f;
            n_ = n;
            grain_ = std::max(1ll, grain);
            next_.store(0);
            busy_ = nt_ - 1;
            gen_++;
        }
        cv_.notify_all();
        work(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return busy_ == 0; });
        job_ = nullptr;
    }

private:
    void work(int t) {
        for (;;) {
            const long long b = next_.fetch_add(grain_);
            if (b >= n_) break;
            (*job_)(t, b, std::min(n_, b + grain_));
        }
    }
    void loop(int t) {
        unsigned long long seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work(t);
            std::lock_guard<std::mutex> lk(mu_);
            if (--busy_ == 0) done_cv_.notify_all();
        }
    }
    int nt_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int, long long, long long)> *job_ = nullptr;
    long long n_ = 0, grain_ = 1;
    std::atomic<long long> next_{0};
    int busy_ = 0;
    unsigned long long gen_ = 0;
    bool stop_ = false;
};

static inline bool atomic_min(int32_t *p, int32_t v) {
    int32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < cur)
        if (__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return true;
    return false;
}

struct Graph {
    int32_t n = 0;
    int64_t m = 0;
    bool symmetric = false;
    std::vector<int32_t> rp, col, irp, icol;  // out-CSR and (directed) its transpose
    std::vector<uint32_t> w;
    const int32_t *in_rp() const { return symmetric ? rp.data() : irp.data(); }
    const int32_t *in_col() const { return symmetric ? col.data() : icol.data(); }
};

static int threads_for(int32_t requested) {
    if (requested > 0) return requested;
    const unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)hc : 1;
}

// ---- BFS ------------------------------------------------------------------------------
static void bfs(const Graph &g, int32_t src, Pool &pool, int32_t *depth) {
    const int n = g.n;
    for (int v = 0; v < n; v++) depth[v] = -1;
    depth[src] = 0;
    std::vector<int32_t> front{src}, next;
    std::vector<std::vector<int32_t>> local(pool.size());
    const int32_t *irp = g.in_rp(), *icol = g.in_col();
    for (int level = 0; !front.empty(); level++) {
        for (auto &l : local) l.clear();
        if ((long long)front.size() * 20 > n) {
            // bottom-up: every unvisited vertex looks for a parent in the frontier
            pool.run(n, 4096, [&](int t, long long b, long long e) {
                for (long long v = b; v < e; v++) {
                    if (depth[v] >= 0) continue;
                    for (int32_t k = irp[v]; k < irp[v + 1]; k++)
                        if (__atomic_load_n(&depth[icol[k]], __ATOMIC_RELAXED) == level) {
                            __atomic_store_n(&depth[v], level + 1, __ATOMIC_RELAXED);
                            local[t].push_back((int32_t)v);
                            break;
                        }
                }
            });
        } else {
            pool.run((long long)front.size(), 64, [&](int t, long long b, long long e) {
                for (long long i = b; i < e; i++) {
                    const int32_t u = front[i];
                    for (int32_t k = g.rp[u]; k < g.rp[u + 1]; k++) {
                        int32_t exp = -1;
                        const int32_t v = g.col[k];
                        if (__atomic_load_n(&depth[v], __ATOMIC_RELAXED) == -1 &&
                            __atomic_compare_exchange_n(&depth[v], &exp, level + 1, false, __ATOMIC_RELAXED,
                                                        __ATOMIC_RELAXED))
                            local[t].push_back(v);
                    }
                }
            });
        }
        next.clear();
        for (auto &l : local) next.insert(next.end(), l.begin(), l.end());
        front.swap(next);
    }
}

// ---- delta-stepping SSSP ----------------------------------------------------------------------
static void sssp(const Graph &g, int32_t src, int32_t delta, Pool &pool, int32_t *dist, bool *overflow) {
    const int n = g.n;
    for (int v = 0; v < n; v++) dist[v] = INT_MAX;
    dist[src] = 0;
    std::vector<std::vector<int32_t>> buckets(1);
    buckets[0].push_back(src);
    std::vector<std::vector<std::pair<long long, int32_t>>> local(pool.size());
    std::atomic<bool> ovf{false};
    std::vector<int32_t> cur;
    for (size_t k = 0; k < buckets.size(); k++) {
        while (!buckets[k].empty()) {
            cur.swap(buckets[k]);
            buckets[k].clear();
            for (auto &l : local) l.clear();
            pool.run((long long)cur.size(), 64, [&](int t, long long b, long long e) {
                for (long long i = b; i < e; i++) {
                    const int32_t u = cur[i];
                    const int32_t du = __atomic_load_n(&dist[u], __ATOMIC_RELAXED);
                    if ((long long)du / delta != (long long)k) continue;  // moved to an earlier bucket: stale
                    for (int32_t e2 = g.rp[u]; e2 < g.rp[u + 1]; e2++) {
                        const long long nd = (long long)du + g.w[e2];
                        const int32_t v = g.col[e2];
                        if (nd > (long long)INT_MAX - 1) {
                            if (__atomic_load_n(&dist[v], __ATOMIC_RELAXED) == INT_MAX) ovf = true;
                            continue;
                        }
                        if (atomic_min(&dist[v], (int32_t)nd)) local[t].emplace_back(nd / delta, v);
                    }
                }
            });
            for (auto &l : local)
                for (auto &bv : l) {
                    if ((size_t)bv.first >= buckets.size()) buckets.resize((size_t)bv.first + 1);
                    buckets[(size_t)bv.first].push_back(bv.second);
                }
        }
    }
    if (ovf) {
        // a vertex left unreached next to a reached one has a distance beyond
        // INT32_MAX-1 (every relaxation into it was unrepresentable)
        for (int v = 0; v < n && !*overflow; v++)
            if (dist[v] == INT_MAX)
                for (int32_t e = g.in_rp()[v]; e < g.in_rp()[v + 1]; e++)
                    if (dist[g.in_col()[e]] != INT_MAX) { *overflow = true; break; }
    }
}

// ---- CC --------------------------------------------------------------------------------------
static void cc(const Graph &g, Pool &pool, int32_t *label) {
    const int n = g.n;
    for (int v = 0; v < n; v++) label[v] = v;
    for (;;) {
        std::atomic<bool> changed{false};
        pool.run(n, 1024, [&](int, long long b, long long e) {
            bool ch = false;
            for (long long u = b; u < e; u++)
                for (int32_t k = g.rp[u]; k < g.rp[u + 1]; k++) {
                    const int32_t v = g.col[k];
                    if (v < u) continue;
                    const int32_t lu = __atomic_load_n(&label[u], __ATOMIC_RELAXED);
                    const int32_t lv = __atomic_load_n(&label[v], __ATOMIC_RELAXED);
                    if (lu == lv) continue;
                    ch |= atomic_min(&label[std::max(lu, lv)], std::min(lu, lv));
                }
            if (ch) changed = true;
        });
        pool.run(n, 4096, [&](int, long long b, long long e) {
            for (long long v = b; v < e; v++) {
                int32_t l = __atomic_load_n(&label[v], __ATOMIC_RELAXED);
                for (;;) {
                    const int32_t ll = __atomic_load_n(&label[l], __ATOMIC_RELAXED);
                    if (ll == l) break;
                    l = ll;
                }
                __atomic_store_n(&label[v], l, __ATOMIC_RELAXED);
            }
        });
        if (!changed) break;
    }
}

// ---- PageRank ---------------------------------------------------------------------------------
static void pagerank(const Graph &g, float damping, int iters, bool dangling, Pool &pool, float *rank_out) {
    const int n = g.n;
    std::vector<float> contrib(n), next(n);
    const int32_t *irp = g.in_rp(), *icol = g.in_col();
    auto outdeg = [&](int v) { return g.rp[v + 1] - g.rp[v]; };
    const float r0 = (float)(1.0 / (double)n);
    double D = 0;
    for (int v = 0; v < n; v++) {
        contrib[v] = outdeg(v) > 0 ? r0 / (float)outdeg(v) : 0.f;
        if (outdeg(v) == 0) D += (double)r0;
        rank_out[v] = r0;
    }
    constexpr int chunks = 1024;  // fixed: the dangling sum's order must not depend on the threads
    std::vector<double> dpart(chunks);
    for (int t = 0; t < iters; t++) {
        const double base = (1.0 - damping) / (double)n + (double)damping * (dangling ? D : 0.0) / (double)n;
        pool.run(n, 2048, [&](int, long long b, long long e) {
            for (long long v = b; v < e; v++) {
                double s = 0.0;
                for (int32_t k = irp[v]; k < irp[v + 1]; k++) s += (double)contrib[icol[k]];
                next[v] = (float)(base + (double)damping * s);
            }
        });
        // contributions and the next round's dangling mass, in a fixed order
        const long long per = ((long long)n + chunks - 1) / chunks;
        pool.run(chunks, 1, [&](int, long long b, long long e) {
            for (long long c = b; c < e; c++) {
                double dl = 0;
                const long long lo = c * per, hi = std::min<long long>(n, lo + per);
                for (long long v = lo; v < hi; v++) {
                    const int d = outdeg((int)v);
                    contrib[v] = d > 0 ? next[v] / (float)d : 0.f;
                    if (d == 0) dl += (double)next[v];
                }
                dpart[c] = dl;
            }
        });
        D = 0;
        for (double x : dpart) D += x;
        std::memcpy(rank_out, next.data(), sizeof(float) * (size_t)n);
    }
}

// ---- BC ---------------------------------------------------------------------------------------------
static void bc(const Graph &g, int32_t src, Pool &pool, uint64_t *sigma, float *delta_out, bool *overflow) {
    const int n = g.n;
    std::vector<int32_t> depth(n, -1);
    std::vector<double> delta(n, 0.0);
    for (int v = 0; v < n; v++) sigma[v] = 0;
    depth[src] = 0;
    sigma[src] = 1;
    std::vector<std::vector<int32_t>> levels{{src}};
    std::vector<std::vector<int32_t>> local(pool.size());
    std::atomic<bool> ovf{false};
    const int32_t *irp = g.in_rp(), *icol = g.in_col();
    // forward: discover the next level top-down, then sum the path counts of
    // each new vertex over its parents (a pull, so no atomics on sigma)
    for (int L = 0; !levels[L].empty(); L++) {
        for (auto &l : local) l.clear();
        const auto &F = levels[L];
        pool.run((long long)F.size(), 64, [&](int t, long long b, long long e) {
            for (long long i = b; i < e; i++)
                for (int32_t k = g.rp[F[i]]; k < g.rp[F[i] + 1]; k++) {
                    int32_t exp = -1;
                    const int32_t v = g.col[k];
                    if (__atomic_load_n(&depth[v], __ATOMIC_RELAXED) == -1 &&
                        __atomic_compare_exchange_n(&depth[v], &exp, L + 1, false, __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED))
                        local[t].push_back(v);
                }
        });
        std::vector<int32_t> nextl;
        for (auto &l : local) nextl.insert(nextl.end(), l.begin(), l.end());
        pool.run((long long)nextl.size(), 64, [&](int, long long b, long long e) {
            for (long long i = b; i < e; i++) {
                const int32_t v = nextl[i];
                uint64_t s = 0;
                for (int32_t k = irp[v]; k < irp[v + 1]; k++) {
                    const int32_t u = icol[k];
                    if (depth[u] == L) {
                        if (s + sigma[u] < s) ovf = true;
                        s += sigma[u];
                    }
                }
                sigma[v] = s;
            }
        });
        levels.push_back(std::move(nextl));
    }
    // backward: deepest level first; each vertex sums over its successors
    for (int L = (int)levels.size() - 2; L >= 0; L--) {
        const auto &F = levels[L];
        pool.run((long long)F.size(), 64, [&](int, long long b, long long e) {
            for (long long i = b; i < e; i++) {
                const int32_t v = F[i];
                double acc = 0.0;
                for (int32_t k = g.rp[v]; k < g.rp[v + 1]; k++) {
                    const int32_t w = g.col[k];
                    if (depth[w] == L + 1) acc += ((double)sigma[v] / (double)sigma[w]) * (1.0 + delta[w]);
                }
                delta[v] = v == src ? 0.0 : acc;
            }
        });
    }
    for (int v = 0; v < n; v++) delta_out[v] = (float)delta[v];
    *overflow = ovf;
}

}  // namespace cpu
}  // namespace gg

using namespace gg;

struct gg_cpu_graph {
    cpu::Graph g;
};

namespace {
template <class Fn>
gg_status cguard(Fn &&fn) {
    try {
        fn();
        g_last_error.clear();
        return GG_OK;
    } catch (const cpu::Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GG_ERR_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GG_ERR_INVALID_ARG;
    }
}

const cpu::Graph &checked(const gg_cpu_graph *g) {
    cpu::require(g != nullptr, GG_ERR_INVALID_ARG, "graph is NULL");
    return g->g;
}
}  // namespace

extern "C" {

gg_status gg_cpu_graph_create(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                              uint32_t flags, gg_cpu_graph **out) {
    return cguard([&] {
        cpu::require(out != nullptr, GG_ERR_INVALID_ARG, "out is NULL");
        cpu::require(n >= 1 && m >= 0 && m < (1ll << 31), GG_ERR_INVALID_ARG, "n must be >= 1 and 0 <= m < 2^31");
        cpu::require(row_ptr != nullptr && (m == 0 || col != nullptr), GG_ERR_INVALID_ARG, "NULL CSR array");
        cpu::require((flags & GG_INPUT_DEVICE) == 0, GG_ERR_INVALID_ARG, "the CPU backend takes host arrays");
        cpu::require(row_ptr[0] == 0 && row_ptr[n] == m, GG_ERR_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n] m");
        auto h = std::make_unique<gg_cpu_graph>();
        cpu::Graph &g = h->g;
        g.n = n;
        g.m = m;
        g.symmetric = (flags & GG_SYMMETRIC) != 0;
        g.rp.assign(row_ptr, row_ptr + n + 1);
        g.col.assign(col, col + m);
        for (int32_t v = 0; v < n; v++) {
            cpu::require(g.rp[v + 1] >= g.rp[v], GG_ERR_INVALID_ARG, "row_ptr not monotone");
            if (flags & GG_VALIDATE)
                for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
                    cpu::require(g.col[e] >= 0 && g.col[e] < n && g.col[e] != v, GG_ERR_INVALID_ARG,
                                 "column out of range or self-loop");
                    cpu::require(e == g.rp[v] || g.col[e] > g.col[e - 1], GG_ERR_INVALID_ARG, "row not ascending");
                }
        }
        if (w) g.w.assign(w, w + m);
        if (!g.symmetric) {  // the transpose, in-rows ascending (stable counting sort)
            g.irp.assign((size_t)n + 1, 0);
            g.icol.resize((size_t)m);
            for (int64_t e = 0; e < m; e++) g.irp[(size_t)g.col[e] + 1]++;
            for (int32_t v = 0; v < n; v++) g.irp[(size_t)v + 1] += g.irp[v];
            std::vector<int32_t> cur(g.irp.begin(), g.irp.end() - 1);
            for (int32_t u = 0; u < n; u++)
                for (int64_t e = g.rp[u]; e < g.rp[u + 1]; e++) g.icol[(size_t)cur[g.col[e]]++] = u;
        }
        *out = h.release();
    });
}

gg_status gg_cpu_graph_destroy(gg_cpu_graph *g) {
    delete g;
    return GG_OK;
}

gg_status gg_cpu_bfs(gg_cpu_graph *cg, int32_t src, int32_t nthreads, int32_t *depth) {
    return cguard([&] {
        const cpu::Graph &g = checked(cg);
        cpu::require(src >= 0 && src < g.n && depth, GG_ERR_INVALID_ARG, "bad source or NULL output");
        cpu::Pool pool(cpu::threads_for(nthreads));
        cpu::bfs(g, src, pool, depth);
    });
}

gg_status gg_cpu_sssp(gg_cpu_graph *cg, int32_t src, int32_t delta, int32_t nthreads, int32_t *dist) {
    return cguard([&] {
        const cpu::Graph &g = checked(cg);
        cpu::require(src >= 0 && src < g.n && dist, GG_ERR_INVALID_ARG, "bad source or NULL output");
        cpu::require(!g.w.empty() || g.m == 0, GG_ERR_INVALID_ARG, "SSSP needs edge weights");
        cpu::require(delta >= 1, GG_ERR_INVALID_ARG, "delta must be >= 1");
        cpu::Pool pool(cpu::threads_for(nthreads));
        bool ovf = false;
        cpu::sssp(g, src, delta, pool, dist, &ovf);
        cpu::require(!ovf, GG_ERR_OVERFLOW, "a shortest-path distance exceeds INT32_MAX-1");
    });
}

gg_status gg_cpu_cc(gg_cpu_graph *cg, int32_t nthreads, int32_t *label) {
    return cguard([&] {
        const cpu::Graph &g = checked(cg);
        cpu::require(label != nullptr, GG_ERR_INVALID_ARG, "NULL output");
        cpu::require(g.symmetric, GG_ERR_INVALID_ARG, "CC needs a symmetric graph (GG_SYMMETRIC)");
        cpu::Pool pool(cpu::threads_for(nthreads));
        cpu::cc(g, pool, label);
    });
}

gg_status gg_cpu_pagerank(gg_cpu_graph *cg, float damping, int32_t iters, uint32_t flags, int32_t nthreads,
                          float *rank) {
    return cguard([&] {
        const cpu::Graph &g = checked(cg);
        cpu::require(rank != nullptr && iters >= 0, GG_ERR_INVALID_ARG, "NULL output or iters < 0");
        cpu::require(damping >= 0.f && damping <= 1.f, GG_ERR_INVALID_ARG, "damping must be in [0, 1]");
        cpu::require((flags & ~(uint32_t)GG_PR_NO_DANGLING) == 0, GG_ERR_INVALID_ARG, "unknown PageRank flags");
        cpu::Pool pool(cpu::threads_for(nthreads));
        cpu::pagerank(g, damping, iters, (flags & GG_PR_NO_DANGLING) == 0, pool, rank);
    });
}

gg_status gg_cpu_bc(gg_cpu_graph *cg, int32_t src, int32_t nthreads, uint64_t *sigma, float *delta) {
    return cguard([&] {
        const cpu::Graph &g = checked(cg);
        cpu::require(src >= 0 && src < g.n && sigma && delta, GG_ERR_INVALID_ARG, "bad source or NULL output");
        cpu::Pool pool(cpu::threads_for(nthreads));
        bool ovf = false;
        cpu::bc(g, src, pool, sigma, delta, &ovf);
        cpu::require(!ovf, GG_ERR_OVERFLOW, "a shortest-path count exceeds 2^64-1");
    });
}

}  // extern "C"
