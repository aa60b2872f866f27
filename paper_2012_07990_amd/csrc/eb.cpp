// EdgeBlocking preprocessing (GPU-Specific Optimizations section, the
// Algorithm for preprocessing the input graph): the COO edge list is counted
// per destination segment floor(dst / N), an exclusive prefix sum gives every
// segment's start, and a second pass scatters each edge to its segment's
// cursor -- a stable counting sort, so sources stay ascending inside a
// segment. Runs once per (graph, N) on the host; the blocked COO is uploaded
// and owned by the graph. The paper's edge-processing algorithm reads
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
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)m);
    GG_HIP(hipMemcpyAsync(rp.data(), G.row_ptr.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, c.s));
    if (m) GG_HIP(hipMemcpyAsync(col.data(), G.col.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, c.s));
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
    for (int32_t u = 0; u < n; u++) {
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            const long long i = cursor[col[e] / N]++;
            osrc[i] = u;
            odst[i] = col[e];
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
    GG_HIP(hipStreamSynchronize(c.s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(G.mu);
    if (!G.eb.count(N)) G.eb[N] = std::move(b);
    return ms;
}

}  // namespace gg
