// Host launchers for the frontier utility kernels (conversions, compaction,
// counting, scans, fills) and the graph/workspace objects shared by the
// algorithm drivers.
#pragma once

#include <map>
#include <utility>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace gg {

// ---- launch bookkeeping ---------------------------------------------------------
struct Ctx {
    hipStream_t s;
    int launches = 0;
    unsigned long long *edge_counter = nullptr;  // device, null unless counting
    int num_cus = 256;
};

// Event timing of one kernel's launches (GG_STATS_TIME_KERNELS).
struct KernelTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    void begin() {
        if (!on) return;
        hipEvent_t a, b;
        GG_HIP(hipEventCreate(&a));
        GG_HIP(hipEventCreate(&b));
        ev.emplace_back(a, b);
        GG_HIP(hipEventRecord(a, s));
    }
    void end() {
        if (!on) return;
        GG_HIP(hipEventRecord(ev.back().second, s));
    }
    // total milliseconds (synchronises); releases the events
    double total() {
        double t = 0;
        for (auto &p : ev) {
            GG_HIP(hipEventSynchronize(p.second));
            float ms = 0;
            GG_HIP(hipEventElapsedTime(&ms, p.first, p.second));
            t += ms;
        }
        for (auto &p : ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        ev.clear();
        return t;
    }
    ~KernelTimer() {
        for (auto &p : ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
};

// ---- device buffers ------------------------------------------------------------------
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    bool fixed = false;  // borrowed memory: never freed, never grown
    ~DevBuf() { release(); }
    void release() {
        if (p && !fixed) (void)hipFree(p);
        p = nullptr;
        n = 0;
        fixed = false;
    }
    // use `count` elements at `ptr` (owned elsewhere); a later ensure() past
    // them throws instead of allocating
    void borrow(T *ptr, size_t count) {
        release();
        p = ptr;
        n = count;
        fixed = true;
    }
    // device bytes held
    size_t bytes() const { return p && !fixed ? (n ? n : 1) * sizeof(T) : 0; }
    // grow-only allocation (contents not preserved)
    void ensure(size_t count) {
        if (count <= n && p) return;
        require(!fixed, GG_ERR_INVALID_ARG, "a borrowed (no-allocation) workspace buffer is too small");
        release();
        size_t bytes = (count ? count : 1) * sizeof(T);
        GG_HIP(hipMalloc(&p, bytes));
        n = count;
    }
};

template <class T>
struct HostPinned {
    T *p = nullptr;
    size_t n = 0;
    bool fixed = false;  // borrowed host memory (not pinned by this object)
    HostPinned() = default;
    HostPinned(const HostPinned &) = delete;
    ~HostPinned() {
        if (p && !fixed) (void)hipHostFree(p);
    }
    void borrow(T *ptr, size_t count) {
        if (p && !fixed) (void)hipHostFree(p);
        p = ptr;
        n = count;
        fixed = true;
    }
    void ensure(size_t count) {
        if (count <= n && p) return;
        require(!fixed, GG_ERR_INVALID_ARG, "a borrowed (no-allocation) host buffer is too small");
        if (p) (void)hipHostFree(p);
        p = nullptr;
        GG_HIP(hipHostMalloc(&p, (count ? count : 1) * sizeof(T), hipHostMallocDefault));
        n = count;
    }
};

// ---- per-query workspace (frontier buffers reused across iterations and calls:
// nothing is allocated inside a traversal loop) ----------------------------------
struct Workspace {
    DevBuf<int32_t> q[2];                 // sparse queues
    DevBuf<int32_t> counters;             // small device counters
    DevBuf<uint8_t> boolmap[2];           // dense boolmaps (n, rounded up)
    DevBuf<unsigned long long> bitmap[2]; // dense bitmaps (ceil(n/64))
    DevBuf<int32_t> tags;                 // monotonic dedup counters
    DevBuf<unsigned long long> dedup_bits;
    DevBuf<unsigned> dedup_bytes;
    DevBuf<int32_t> bins;                 // TWC tiers (3 x cap)
    DevBuf<long long> scan;               // STRICT degree scan (cap + 1)
    DevBuf<long long> scan_part;          // scan partials
    DevBuf<int32_t> aux_i32[4];           // algorithm-specific
    DevBuf<unsigned long long> aux_u64[3];
    DevBuf<float> aux_f32[3];
    DevBuf<double> aux_f64[2];
    DevBuf<uint8_t> member;               // EDGE_ONLY input-frontier membership map
    DevBuf<float> pr_contrib[2];  // PageRank
    DevBuf<float> pr_hot[2];      // PageRank STRICT: contributions of the LDS-cached sources
    DevBuf<double> pr_acc, pr_head, pr_tail;
    DevBuf<double> pr_partial, pr_dangling;
    DevBuf<unsigned long long> ms_sigma;  // multi-source BC path counts (vertex-major)
    DevBuf<unsigned> barrier;             // grid barrier state for fused kernels
    HostPinned<int32_t> h_i32;            // pinned readback slots
    HostPinned<long long> h_i64;
    size_t lease_bytes = 0;               // bytes() when it was last leased from the pool

    // device bytes held by every buffer above
    size_t bytes() const {
        size_t b = counters.bytes() + tags.bytes() + dedup_bits.bytes() + dedup_bytes.bytes() + bins.bytes() +
                   scan.bytes() + scan_part.bytes() + member.bytes() + pr_acc.bytes() + pr_head.bytes() +
                   pr_tail.bytes() + pr_partial.bytes() + pr_dangling.bytes() + ms_sigma.bytes() + barrier.bytes();
        for (int i = 0; i < 2; i++)
            b += q[i].bytes() + boolmap[i].bytes() + bitmap[i].bytes() + aux_f64[i].bytes() + pr_contrib[i].bytes() +
                 pr_hot[i].bytes();
        for (int i = 0; i < 3; i++) b += aux_u64[i].bytes() + aux_f32[i].bytes();
        for (int i = 0; i < 4; i++) b += aux_i32[i].bytes();
        return b;
    }
};

// ---- graph ------------------------------------------------------------------------------
struct EdgeBlocked {
    DevBuf<int32_t> src, dst;
    DevBuf<uint32_t> w;  // the edges' weights in blocked order (weighted graphs)
    std::vector<long long> seg_start;  // host copy, S + 1 entries
    int32_t seg_vertices = 0;
};

// PULL EdgeBlocking: the CSR split by source segment [s*N, (s+1)*N); each
// segment is a CSR over all destinations (rows keep their ascending order).
struct PullBlocked {
    int32_t N = 0;
    int S = 0;
    DevBuf<int32_t> rp;    // S x (n+1) row offsets (unused when S == 1)
    DevBuf<int32_t> col;   // m sources, segment-major (unused when S == 1)
    const int32_t *rp_ptr = nullptr, *col_ptr = nullptr;  // the layout in use
    std::vector<long long> m_s, col_base;
    DevBuf<int32_t> chunk_rows;            // per segment: owner rows of each chunk's first/last edge
    std::vector<long long> chunk_base, nchunks;
    int hot_k = 0;                         // sources per segment cached in LDS (slots per segment)
    DevBuf<int32_t> hot_slot;              // n: segment*hot_k + slot of a cached source, else -1
    DevBuf<int32_t> hcol;                  // col_ptr's layout with cached sources as ~slot
};

// CC EdgeBlocking: the upper-triangle pair list grouped by destination
// segment floor(v / N), CSR order kept inside a segment
struct BlockedPairs {
    int32_t N = 0;
    DevBuf<int2> pairs;
    std::vector<long long> seg_start;  // S + 1 entries
};

struct Graph {
    int32_t n = 0;
    int64_t m = 0;
    bool symmetric = false;
    bool has_weights = false;
    DevBuf<int32_t> row_ptr, col, coo_src;
    DevBuf<int2> upper;        // symmetric graphs: every undirected edge once as (u, v), u < v, CSR order
    int64_t m_upper = 0;
    DevBuf<int32_t> in_rp, in_col;  // directed graphs: the transpose (in-edges), built for PULL
    DevBuf<uint32_t> w;
    int32_t max_degree = 0;
    std::map<int32_t, std::unique_ptr<EdgeBlocked>> eb;  // per blocking size
    std::map<int32_t, std::unique_ptr<PullBlocked>> pull_eb;  // STRICT pull partitions per segment width
    std::map<int32_t, std::unique_ptr<BlockedPairs>> upper_eb;  // CC pair lists per segment width
    std::map<int, std::pair<gg_schedule, double>> tuned;       // autotuner winners (schedule, ms) per algorithm
    std::map<int, int> placement;                              // measured CPU-or-GPU target per algorithm
    std::mutex mu;
    std::vector<std::unique_ptr<Workspace>> pool;
    size_t leased = 0;  // lease_bytes of the workspaces leased out now
    int device = 0;
    int num_cus = 256;

    DevGraph view() const {
        return DevGraph{n,
                        m,
                        row_ptr.p,
                        col.p,
                        has_weights ? w.p : nullptr,
                        coo_src.p,
                        symmetric ? row_ptr.p : in_rp.p,
                        symmetric ? col.p : in_col.p};
    }
    std::unique_ptr<Workspace> acquire();
    void give_back(std::unique_ptr<Workspace> ws);
    // device bytes held by the pooled workspaces plus those leased out (at
    // their size when leased), and by the derived layouts built so far (COO
    // sources, EdgeBlocked COO, pull blocking)
    size_t pooled_bytes();
    size_t layout_bytes();
    // free pooled workspaces until at most `keep` bytes stay pooled;
    // returns the bytes freed
    size_t trim_pool(size_t keep);
};

// RAII lease of a workspace from the graph's pool
struct Lease {
    Graph &g;
    std::unique_ptr<Workspace> ws;
    explicit Lease(Graph &gr) : g(gr), ws(gr.acquire()) {}
    ~Lease() { g.give_back(std::move(ws)); }
    Workspace *operator->() { return ws.get(); }
    Workspace &operator*() { return *ws; }
};

// ---- utility launchers (kernels in frontier_ops.hip) ----------------------------------
void fill_i32(Ctx &c, int32_t *p, long long n, int32_t v);
void fill_u8(Ctx &c, uint8_t *p, long long n, uint8_t v);
void fill_u64(Ctx &c, unsigned long long *p, long long n, unsigned long long v);
void fill_f32(Ctx &c, float *p, long long n, float v);
void fill_f64(Ctx &c, double *p, long long n, double v);
// queue -> dense map (map must be cleared first)
void queue_to_boolmap(Ctx &c, const int32_t *q, int count, uint8_t *map);
void queue_to_bitmap(Ctx &c, const int32_t *q, int count, unsigned long long *map);
// dense map -> dense map (writes every word/byte of dst)
void boolmap_to_bitmap(Ctx &c, const uint8_t *src, int n, unsigned long long *dst);
void bitmap_to_boolmap(Ctx &c, const unsigned long long *src, int n, uint8_t *dst);
// dense map -> queue; count must be zeroed by the caller (device int)
void boolmap_to_queue(Ctx &c, const uint8_t *map, int n, int32_t *q, int32_t *count);
void bitmap_to_queue(Ctx &c, const unsigned long long *map, int n, int32_t *q, int32_t *count);
// population counts into a device int (zeroed by the caller)
void count_boolmap(Ctx &c, const uint8_t *map, int n, int32_t *count);
void count_bitmap(Ctx &c, const unsigned long long *map, int n, int32_t *count);
// exclusive scan of the degrees of q[0..count) into scan[0..count] (int64);
// zeroes *zero too when it is not null (one or two launches)
void degree_scan(Ctx &c, const DevGraph &g, const int32_t *q, int count, long long *scan,
                 long long *partials, int32_t *zero = nullptr);
size_t degree_scan_partials(int count);
// in place: data[0..n) counts -> data[0..n] exclusive offsets (int32 totals)
void exclusive_scan_i32(Ctx &c, int32_t *data, int n, long long *partials);
size_t exclusive_scan_partials(int n);

// device -> pinned host readback of one int, then stream sync
int32_t read_i32(Ctx &c, const int32_t *dev, int32_t *pinned);

}  // namespace gg
