// EdgeBlocking preprocessing (GPU-Specific Optimizations section, the
// Algorithm for preprocessing the input graph): the COO edge list is counted
// per destination segment floor(dst / N), an exclusive prefix sum gives every
// segment's start, and a second pass scatters each edge to its segment's
// cursor -- a stable counting sort, so sources stay ascending inside a
// segment. Runs once per (graph, N) on the host; the blocked COO (and, on a
// weighted graph, the weights in the same order) is uploaded and owned by
// the graph. The paper's edge-processing algorithm reads
// segmentStart[segIdx-1] as the start of segment segIdx; here seg_start has
// S+1 entries and segment s is [seg_start[s], seg_start[s+1]).
#include <hip/hip_runtime.h>

#include <chrono>
#include <vector>

#include "algos.hpp"

namespace gg {

double edgeblock_prepare(Ctx &c, Graph &G, int32_t N) {
    require(N >= 1, GG_ERR_INVALID_ARG, "blocking size must be >= 1");
    {
        std::lock_guard<std::mutex> lk(G.mu);
        if (G.eb.count(N)) return 0.0;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int32_t n = G.n;
    const int64_t m = G.m;
    const bool weighted = G.has_weights && m > 0;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)m);
    std::vector<uint32_t> w(weighted ? (size_t)m : 0);
    GG_HIP(hipMemcpyAsync(rp.data(), G.row_ptr.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, c.s));
    if (m) GG_HIP(hipMemcpyAsync(col.data(), G.col.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, c.s));
    if (weighted) GG_HIP(hipMemcpyAsync(w.data(), G.w.p, sizeof(uint32_t) * m, hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    const int64_t S = ((int64_t)n + N - 1) / N;
    std::vector<long long> count((size_t)S + 1, 0), start((size_t)S + 1, 0);
    for (int64_t e = 0; e < m; e++) count[col[e] / N]++;
    long long run = 0;
    for (int64_t s = 0; s <= S; s++) {
        start[s] = run;
        run += count[s];
    }
    std::vector<long long> cursor(start);
    std::vector<int32_t> osrc((size_t)m), odst((size_t)m);
    std::vector<uint32_t> ow(weighted ? (size_t)m : 0);
    for (int32_t u = 0; u < n; u++) {
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            const long long i = cursor[col[e] / N]++;
            osrc[i] = u;
            odst[i] = col[e];
            if (weighted) ow[i] = w[e];
        }
    }
    auto b = std::make_unique<EdgeBlocked>();
    b->seg_vertices = N;
    b->seg_start = start;
    b->src.ensure((size_t)(m > 0 ? m : 1));
    b->dst.ensure((size_t)(m > 0 ? m : 1));
    if (m) {
        GG_HIP(hipMemcpyAsync(b->src.p, osrc.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c.s));
        GG_HIP(hipMemcpyAsync(b->dst.p, odst.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c.s));
    }
    if (weighted) {
        b->w.ensure((size_t)m);
        GG_HIP(hipMemcpyAsync(b->w.p, ow.data(), sizeof(uint32_t) * m, hipMemcpyHostToDevice, c.s));
    }
    GG_HIP(hipStreamSynchronize(c.s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(G.mu);
    if (!G.eb.count(N)) G.eb[N] = std::move(b);
    return ms;
}

// In-edges of a directed graph for PULL traversals (the configDirection
// PULL choice reads the sources of each destination): the transpose of the
// CSR by a stable counting sort over destinations, so each in-row keeps its
// sources ascending. Runs once per graph on the host, like the preprocessing
// above; the transpose is uploaded and owned by the graph, published only
// once complete. Symmetric graphs read their own CSR.
void ensure_transpose(Ctx &c, Graph &G) {
    if (G.symmetric) return;
    std::lock_guard<std::mutex> lk(G.mu);
    if (G.in_rp.p) return;
    const int32_t n = G.n;
    const int64_t m = G.m;
    const bool weighted = G.has_weights && m > 0;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)m);
    std::vector<uint32_t> w(weighted ? (size_t)m : 0);
    GG_HIP(hipMemcpyAsync(rp.data(), G.row_ptr.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, c.s));
    if (m) GG_HIP(hipMemcpyAsync(col.data(), G.col.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, c.s));
    if (weighted) GG_HIP(hipMemcpyAsync(w.data(), G.w.p, sizeof(uint32_t) * m, hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    std::vector<int32_t> irp((size_t)n + 1, 0), icol((size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; e++) irp[(size_t)col[e] + 1]++;
    for (int32_t v = 0; v < n; v++) irp[(size_t)v + 1] += irp[v];
    std::vector<int32_t> cursor(irp.begin(), irp.end() - 1);
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) icol[(size_t)cursor[col[e]]++] = u;
    DevBuf<int32_t> drp, dcol;
    drp.ensure((size_t)n + 1);
    dcol.ensure((size_t)(m > 0 ? m : 1));
    GG_HIP(hipMemcpyAsync(drp.p, irp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, c.s));
    if (m) GG_HIP(hipMemcpyAsync(dcol.p, icol.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    std::swap(G.in_rp.p, drp.p);
    std::swap(G.in_rp.n, drp.n);
    std::swap(G.in_col.p, dcol.p);
    std::swap(G.in_col.n, dcol.n);
}

}  // namespace gg
