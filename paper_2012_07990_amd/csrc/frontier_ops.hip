// Frontier utility kernels: fills, representation conversions, wave-ballot
// compaction of dense maps into sparse queues, population counts and the
// device-wide degree scan used by STRICT load balancing.
#include "frontier.hpp"
#include "ops.hpp"

namespace gg {

// ---- fills (kernels rather than memset nodes, so callers may capture them) ----
template <class T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, long long n, T v) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <class T>
static void fill(Ctx &c, T *p, long long n, T v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n, kBlock, 8192)), dim3(kBlock), 0, c.s, p, n, v);
    GG_CHECK_LAUNCH();
    c.launches++;
}
void fill_i32(Ctx &c, int32_t *p, long long n, int32_t v) { fill(c, p, n, v); }
void fill_u8(Ctx &c, uint8_t *p, long long n, uint8_t v) {
    // byte maps are filled a word at a time when aligned
    if (((uintptr_t)p & 3) == 0 && (n & 3) == 0) {
        const uint32_t w = 0x01010101u * v;
        fill(c, reinterpret_cast<uint32_t *>(p), n / 4, w);
    } else {
        fill(c, p, n, v);
    }
}
void fill_u64(Ctx &c, unsigned long long *p, long long n, unsigned long long v) { fill(c, p, n, v); }
void fill_f32(Ctx &c, float *p, long long n, float v) { fill(c, p, n, v); }
void fill_f64(Ctx &c, double *p, long long n, double v) { fill(c, p, n, v); }

// ---- queue -> dense ---------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_queue_to_boolmap(const int32_t *q, int count, uint8_t *map) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) map[q[i]] = 1;
}
__global__ __launch_bounds__(kBlock) void k_queue_to_bitmap(const int32_t *q, int count,
                                                            unsigned long long *map) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
        const int v = q[i];
        atomic_or_u64(&map[v >> 6], 1ull << (v & 63));
    }
}
void queue_to_boolmap(Ctx &c, const int32_t *q, int count, uint8_t *map) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_queue_to_boolmap, dim3(blocks_for(count, kBlock, 8192)), dim3(kBlock), 0, c.s, q,
                       count, map);
    GG_CHECK_LAUNCH();
    c.launches++;
}
void queue_to_bitmap(Ctx &c, const int32_t *q, int count, unsigned long long *map) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_queue_to_bitmap, dim3(blocks_for(count, kBlock, 8192)), dim3(kBlock), 0, c.s, q,
                       count, map);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// ---- dense <-> dense: one lane per vertex, one ballot word per wave ----------------------
__global__ __launch_bounds__(kBlock) void k_boolmap_to_bitmap(const uint8_t *src, int n,
                                                              unsigned long long *dst) {
    const long long stride = (long long)gridDim.x * kBlock;
    const long long nr = ((long long)n + kWave - 1) / kWave * kWave;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < nr; v += stride) {
        const bool on = v < n && src[v];
        const uint64_t word = __ballot(on);
        if (lane_id() == 0) dst[v >> 6] = word;
    }
}
__global__ __launch_bounds__(kBlock) void k_bitmap_to_boolmap(const unsigned long long *src, int n,
                                                              uint8_t *dst) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
        dst[v] = (uint8_t)((src[v >> 6] >> (v & 63)) & 1ull);
}
void boolmap_to_bitmap(Ctx &c, const uint8_t *src, int n, unsigned long long *dst) {
    hipLaunchKernelGGL(k_boolmap_to_bitmap, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, src, n,
                       dst);
    GG_CHECK_LAUNCH();
    c.launches++;
}
void bitmap_to_boolmap(Ctx &c, const unsigned long long *src, int n, uint8_t *dst) {
    hipLaunchKernelGGL(k_bitmap_to_boolmap, dim3(blocks_for(n, kBlock, 16384)), dim3(kBlock), 0, c.s, src, n,
                       dst);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// ---- dense -> queue (ballot compaction staged per workgroup: one global atomic per flush)
__global__ __launch_bounds__(kBlock) void k_boolmap_to_queue(const uint8_t *map, int n, int32_t *q,
                                                             int32_t *count) {
    __shared__ StageLDS s_st;
    if (threadIdx.x == 0) s_st.c = 0;
    __syncthreads();
    OutFrontier o{};
    o.q = q;
    o.count = count;
    o.cap = n;  // a set never exceeds n
    o.overflow = count;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long base = (long long)blockIdx.x * kBlock; base < n; base += stride) {
        const long long v = base + threadIdx.x;
        emit_staged<kCreateFused, kDedupNone>(o, s_st, v < n && map[v], (int)v);
        if ((base / stride) % 8 == 7 || base + stride >= n) emit_flush<kCreateFused>(o, s_st);
    }
}
// one lane per 64-bit word: each lane writes its word's set bits in order;
// one atomic on the queue count per workgroup tile (atomics on one address
// serialise)
__global__ __launch_bounds__(kBlock) void k_bitmap_to_queue(const unsigned long long *map, int nwords,
                                                            int32_t *q, int32_t *count) {
    __shared__ int s_w[kBlock / kWave], s_base;
    const int wib = threadIdx.x / kWave;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long b0 = (long long)blockIdx.x * kBlock; b0 < nwords; b0 += stride) {
        const long long wi = b0 + threadIdx.x;
        unsigned long long word = wi < nwords ? map[wi] : 0ull;
        const int cnt = __popcll(word);
        const int incl = wave_incl_scan(cnt);
        if (lane_id() == kWave - 1) s_w[wib] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; w++) {
            const int x = s_w[w];
            before += w < wib ? x : 0;
            total += x;
        }
        if (threadIdx.x == 0) s_base = total ? atomic_add_i32(count, total) : 0;
        __syncthreads();
        int pos = s_base + before + incl - cnt;
        __syncthreads();  // s_w and s_base are rewritten by the next tile
        while (word) {
            const int b = __ffsll(word) - 1;
            q[pos++] = (int)(wi * 64 + b);
            word &= word - 1;
        }
    }
}
void boolmap_to_queue(Ctx &c, const uint8_t *map, int n, int32_t *q, int32_t *count) {
    // few workgroups, each flushing its staged appends every 8 tiles: the
    // flushes' atomics on the one queue count serialise
    hipLaunchKernelGGL(k_boolmap_to_queue, dim3(blocks_for(n, kBlock * 8, 1024)), dim3(kBlock), 0, c.s, map, n, q,
                       count);
    GG_CHECK_LAUNCH();
    c.launches++;
}
void bitmap_to_queue(Ctx &c, const unsigned long long *map, int n, int32_t *q, int32_t *count) {
    const int nwords = (n + 63) / 64;
    hipLaunchKernelGGL(k_bitmap_to_queue, dim3(blocks_for(nwords, kBlock, 16384)), dim3(kBlock), 0, c.s, map,
                       nwords, q, count);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// ---- population counts ---------------------------------------------------------------------
// One atomic per workgroup on the shared count: atomics on one address
// serialise, and one per wavefront (16K for a 4M-vertex boolmap) made a count
// take ~190 us.
__device__ __forceinline__ void block_add_count(int local, int32_t *count) {
    __shared__ int s_w[kBlock / kWave];
    local = wave_sum(local);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; w++) t += s_w[w];
        if (t) atomic_add_i32(count, t);
    }
}

// non-zero bytes of a 32-bit word
__device__ __forceinline__ int nonzero_bytes(unsigned x) {
    const unsigned zero = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);  // 0x80 per zero byte
    return 4 - __popc(zero);
}

// 16 bytes per lane when the map is 16-byte aligned, the tail byte by byte
__global__ __launch_bounds__(kBlock) void k_count_boolmap(const uint8_t *map, int n, int32_t *count) {
    const long long stride = (long long)gridDim.x * kBlock;
    const long long gid = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nq = (reinterpret_cast<uintptr_t>(map) & 15) == 0 ? n / 16 : 0;
    int local = 0;
    const uint4 *m4 = reinterpret_cast<const uint4 *>(map);
    for (long long i = gid; i < nq; i += stride) {
        const uint4 x = m4[i];
        local += nonzero_bytes(x.x) + nonzero_bytes(x.y) + nonzero_bytes(x.z) + nonzero_bytes(x.w);
    }
    for (long long v = nq * 16 + gid; v < n; v += stride) local += map[v] ? 1 : 0;
    block_add_count(local, count);
}
__global__ __launch_bounds__(kBlock) void k_count_bitmap(const unsigned long long *map, int nwords,
                                                         int32_t *count) {
    const long long stride = (long long)gridDim.x * kBlock;
    int local = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nwords; i += stride)
        local += __popcll(map[i]);
    block_add_count(local, count);
}
void count_boolmap(Ctx &c, const uint8_t *map, int n, int32_t *count) {
    hipLaunchKernelGGL(k_count_boolmap, dim3(blocks_for(((long long)n + 15) / 16, kBlock, 1024)), dim3(kBlock), 0,
                       c.s, map, n, count);
    GG_CHECK_LAUNCH();
    c.launches++;
}
void count_bitmap(Ctx &c, const unsigned long long *map, int n, int32_t *count) {
    const int nwords = (n + 63) / 64;
    hipLaunchKernelGGL(k_count_bitmap, dim3(blocks_for(nwords, kBlock, 1024)), dim3(kBlock), 0, c.s, map,
                       nwords, count);
    GG_CHECK_LAUNCH();
    c.launches++;
}

// ---- device-wide exclusive scan of frontier degrees (reduce, scan partials, apply) -----------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ long long block_sum_ll(long long x, long long *s_tmp) {
    x = wave_sum(x);
    if (lane_id() == 0) s_tmp[threadIdx.x / kWave] = x;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) t += s_tmp[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(DevGraph g, const int32_t *q, int count,
                                                        long long *partials) {
    __shared__ long long s_tmp[kBlock / kWave];
    const long long base = (long long)blockIdx.x * kScanTile;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = base + (long long)k * kBlock + threadIdx.x;
        if (i < count) {
            const int u = q[i];
            s += g.row_ptr[u + 1] - g.row_ptr[u];
        }
    }
    s = block_sum_ll(s, s_tmp);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// single workgroup of 1024 lanes: exclusive scan of the partials in place
__global__ __launch_bounds__(1024) void k_scan_partials(long long *partials, int np) {
    __shared__ long long s_w[1024 / kWave];
    const int per = (np + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(np, lo + per);
    long long s = 0;
    for (int i = lo; i < hi; i++) s += partials[i];
    const long long incl = wave_incl_scan64(s);
    if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = incl;
    __syncthreads();
    long long off = 0;
    for (int w = 0; w < (int)(threadIdx.x / kWave); w++) off += s_w[w];
    long long run = off + incl - s;
    for (int i = lo; i < hi; i++) {
        const long long v = partials[i];
        partials[i] = run;
        run += v;
    }
}

// partials: per-tile degree sums from k_scan_reduce, which each workgroup adds
// up for the tiles before it (scanned false: up to kInlineTiles tiles), or
// their exclusive scan (scanned true), or null for a single tile. zero: a
// counter to clear on the way (the next push's output count).
constexpr int kInlineTiles = 4096;
__global__ __launch_bounds__(kBlock) void k_scan_apply(DevGraph g, const int32_t *q, int count,
                                                       const long long *partials, bool scanned, long long *scan,
                                                       int32_t *zero) {
    __shared__ long long s_w[kBlock / kWave];
    __shared__ long long s_tmp[kBlock / kWave];
    if (zero != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *zero = 0;
    long long off = 0;
    if (partials != nullptr && scanned) {
        off = partials[blockIdx.x];
    } else if (partials != nullptr) {
        long long t = 0;
        for (int j = threadIdx.x; j < (int)blockIdx.x; j += kBlock) t += partials[j];
        off = block_sum_ll(t, s_tmp);
    }
    const long long base = (long long)blockIdx.x * kScanTile;
    // each lane owns kScanItems consecutive entries
    const long long first = base + (long long)threadIdx.x * kScanItems;
    long long vals[kScanItems];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = first + k;
        long long d = 0;
        if (i < count) {
            const int u = q[i];
            d = g.row_ptr[u + 1] - g.row_ptr[u];
        }
        vals[k] = d;
        s += d;
    }
    const long long incl = wave_incl_scan64(s);
    if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = incl;
    __syncthreads();
    for (int w = 0; w < (int)(threadIdx.x / kWave); w++) off += s_w[w];
    long long run = off + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = first + k;
        if (i < count) scan[i] = run;
        if (i == count) scan[i] = run;  // total
        run += vals[k];
    }
    if (count == 0 && blockIdx.x == 0 && threadIdx.x == 0) scan[0] = 0;
}

size_t degree_scan_partials(int count) { return (size_t)(count + kScanTile - 1) / kScanTile + 1; }

void degree_scan(Ctx &c, const DevGraph &g, const int32_t *q, int count, long long *scan,
                 long long *partials, int32_t *zero) {
    // tiles cover [0, count] inclusive so the total lands in scan[count]
    const int tiles = (count + 1 + kScanTile - 1) / kScanTile;
    const bool scanned = tiles > kInlineTiles;
    if (tiles > 1) {
        hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(kBlock), 0, c.s, g, q, count, partials);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
    if (scanned) {
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, c.s, partials, tiles);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kBlock), 0, c.s, g, q, count,
                       (const long long *)(tiles > 1 ? partials : nullptr), scanned, scan, zero);
    GG_CHECK_LAUNCH();
    c.launches++;
}

int32_t read_i32(Ctx &c, const int32_t *dev, int32_t *pinned) {
    GG_HIP(hipMemcpyAsync(pinned, dev, sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GG_HIP(hipStreamSynchronize(c.s));
    return *pinned;
}

}  // namespace gg

namespace gg {

// COO source of every CSR entry: one wavefront per vertex writes its row.
__global__ __launch_bounds__(kBlock) void k_build_coo(const int32_t *row_ptr, int n, int32_t *coo_src) {
    const int wpb = kBlock / kWave;
    for (int v = blockIdx.x * wpb + threadIdx.x / kWave; v < n; v += gridDim.x * wpb) {
        const int end = row_ptr[v + 1];
        for (int e = row_ptr[v] + lane_id(); e < end; e += kWave) coo_src[e] = v;
    }
}

// Built under the graph's lock and completed (stream synchronised) before the
// lock is released: a query on another stream that finds the array already
// present reads a finished array.
void ensure_coo(Ctx &c, Graph &G) {
    std::lock_guard<std::mutex> lk(G.mu);
    if (G.coo_src.p) return;
    G.coo_src.ensure((size_t)G.m);
    if (G.m > 0) {
        hipLaunchKernelGGL(k_build_coo, dim3(blocks_for(G.n, kBlock / kWave, 16384)), dim3(kBlock), 0, c.s,
                           G.row_ptr.p, G.n, G.coo_src.p);
        const hipError_t e = hipGetLastError();
        const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(c.s) : e;
        if (e2 != hipSuccess) {
            G.coo_src.release();
            GG_HIP(e2);
        }
        c.launches++;
    }
}

}  // namespace gg

namespace gg {

// ---- generic in-place exclusive scan of int32 counts: data[0..n) counts ->
// data[0..n] offsets (data[n] = total). Totals must fit in int32.
__global__ __launch_bounds__(kBlock) void k_iscan_reduce(const int32_t *data, int n, long long *partials) {
    __shared__ long long s_tmp[kBlock / kWave];
    const long long base = (long long)blockIdx.x * kScanTile;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = base + (long long)k * kBlock + threadIdx.x;
        if (i < n) s += data[i];
    }
    s = block_sum_ll(s, s_tmp);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_iscan_apply(int32_t *data, int n, const long long *partials) {
    __shared__ long long s_w[kBlock / kWave];
    const long long base = (long long)blockIdx.x * kScanTile;
    const long long first = base + (long long)threadIdx.x * kScanItems;
    long long vals[kScanItems];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = first + k;
        vals[k] = i < n ? data[i] : 0;
        s += vals[k];
    }
    const long long incl = wave_incl_scan64(s);
    if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = incl;
    __syncthreads();
    long long off = partials[blockIdx.x];
    for (int w = 0; w < (int)(threadIdx.x / kWave); w++) off += s_w[w];
    long long run = off + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const long long i = first + k;
        if (i <= n) data[i] = (int32_t)run;
        run += vals[k];
    }
}

void exclusive_scan_i32(Ctx &c, int32_t *data, int n, long long *partials) {
    const int tiles = (n + 1 + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_iscan_reduce, dim3(tiles), dim3(kBlock), 0, c.s, data, n, partials);
    GG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, c.s, partials, tiles);
    GG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_iscan_apply, dim3(tiles), dim3(kBlock), 0, c.s, data, n, partials);
    GG_CHECK_LAUNCH();
    c.launches += 3;
}

size_t exclusive_scan_partials(int n) { return (size_t)(n + 1 + kScanTile - 1) / kScanTile + 1; }

}  // namespace gg
