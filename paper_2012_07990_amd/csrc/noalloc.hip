// BFS entry point that allocates nothing: its workspace (frontier queues,
// dense maps, dedup tags, the STRICT degree scan, the TWC tiers, the grid
// barrier of the persistent form) is carved from a fixed device array, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it).
//
// The array lives in this file as a __device__ symbol, one copy per GPU, held
// until the process ends. Host code never passes the symbol itself: on the
// first call on a device (with that device current) its device address is
// looked up with hipGetSymbolAddress and kept per device; only that address
// reaches kernels and fills. Every call on one GPU shares its copy and leaves
// its contents behind: whatever must start at zero is cleared by the BFS
// driver's fill kernels, and calls that overlap on one GPU race.
#include <mutex>

#include "algos.hpp"
#include "handles.hpp"

namespace gg {

constexpr int32_t kNoAllocMaxN = 1 << 20;                 // largest graph (vertices) it accepts
constexpr size_t kNoAllocScratchBytes = 40ull << 20;      // 40 MiB per GPU
constexpr int kNoAllocMaxDevices = 64;
constexpr size_t kNoAllocBarrierWords = 4096 + 4;         // grid barrier: one word per workgroup + 4

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kNoAllocMaxDevices] = {};
int32_t g_host_slots[kNoAllocMaxDevices][16];  // readback slots (pageable host memory)

// device address of this device's copy of the scratch array
unsigned char *scratch_for(int dev) {
    require(dev >= 0 && dev < kNoAllocMaxDevices, GG_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        require(e == hipSuccess && ptr != nullptr, GG_ERR_DEVICE,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    return g_scratch_ptr[dev];
}

// bump carving of the scratch array (256-byte aligned pieces)
struct Carver {
    unsigned char *base;
    size_t used = 0;
    template <class T>
    void give(DevBuf<T> &b, size_t count) {
        const size_t bytes = (count ? count : 1) * sizeof(T);
        require(used + bytes <= kNoAllocScratchBytes, GG_ERR_INVALID_ARG,
                "no-allocation BFS: the workspace exceeds the fixed scratch array");
        b.borrow(reinterpret_cast<T *>(base + used), count);
        used += (bytes + 255) / 256 * 256;
    }
};

}  // namespace

// Workspace of one BFS over n vertices: every buffer any BFS schedule the
// entry point accepts can ask for, at its largest size.
static void carve_bfs_workspace(Workspace &ws, unsigned char *base, int32_t n) {
    Carver cv{base};
    const size_t nb = ((size_t)n + 255) / 256 * 256;
    for (int i = 0; i < 2; i++) {
        cv.give(ws.q[i], (size_t)n);
        cv.give(ws.boolmap[i], nb);
        cv.give(ws.bitmap[i], nb / 64);
    }
    cv.give(ws.counters, 64);
    cv.give(ws.tags, (size_t)n);
    cv.give(ws.dedup_bits, nb / 64);
    cv.give(ws.dedup_bytes, nb / 4);
    cv.give(ws.bins, (size_t)3 * n);
    cv.give(ws.scan, (size_t)n + 1);
    cv.give(ws.scan_part, degree_scan_partials(n) + kNoAllocBarrierWords);  // also a persistent grid's partials
    cv.give(ws.barrier, kNoAllocBarrierWords);
}

static bool uses_lb(const gg_schedule &s, int lb) {
    return s.s1.load_balance == lb || (s.hybrid && s.s2.load_balance == lb);
}

}  // namespace gg

using namespace gg;

extern "C" gg_status gg_bfs_noalloc(gg_graph *g, int32_t src, const gg_schedule *s, int32_t *depth_dev,
                                    gg_stream_t stream) {
    try {
        require(g != nullptr, GG_ERR_INVALID_ARG, "graph is NULL");
        Graph &G = g->g;
        require(G.n <= kNoAllocMaxN, GG_ERR_INVALID_ARG,
                "no-allocation BFS accepts at most " + std::to_string(kNoAllocMaxN) + " vertices");
        require(src >= 0 && src < G.n, GG_ERR_INVALID_ARG, "source out of range");
        require(depth_dev != nullptr, GG_ERR_INVALID_ARG, "depth is NULL");
        const gg_schedule sc = s ? *s : default_schedule();
        validate_schedule(G, GG_ALGO_BFS, sc);
        require(!uses_lb(sc, GG_LB_EDGE_ONLY), GG_ERR_UNSUPPORTED_SCHEDULE,
                "no-allocation BFS: EDGE_ONLY needs the graph's COO array, which it would allocate");
        require((size_t)4 * G.num_cus + 4 <= kNoAllocBarrierWords, GG_ERR_DEVICE, "too many compute units");
        require(G.symmetric || !schedule_pulls(sc) || G.in_rp.p != nullptr, GG_ERR_UNSUPPORTED_SCHEDULE,
                "no-allocation BFS: PULL on a directed graph needs its transpose, which it would allocate "
                "(run one PULL query through gg_bfs first)");
        int dev = 0;
        GG_HIP(hipGetDevice(&dev));
        require(dev == G.device, GG_ERR_INVALID_ARG, "the graph lives on another device than the current one");
        unsigned char *base = scratch_for(dev);
        Workspace ws;
        carve_bfs_workspace(ws, base, G.n);
        ws.h_i32.borrow(g_host_slots[dev], 16);
        bfs_run_ws(G, ws, src, sc, depth_dev, reinterpret_cast<hipStream_t>(stream), nullptr);
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
