// Host-side frontier bookkeeping shared by the level-synchronous (unfused)
// algorithm drivers: which representation currently holds the frontier,
// double-buffered storage for each representation (reused across iterations,
// never allocated inside the loop), representation conversions and output
// preparation for each creation mode.
#pragma once

#include "traverse.hpp"

namespace gg {

enum Rep : int { kRepQueue = 0, kRepBoolmap = 1, kRepBitmap = 2 };

struct FrontierState {
    Ctx &c;
    Workspace &ws;
    int n;
    long long qcap;
    int rep = kRepQueue;
    int qi = 0, bi = 0, ti = 0;  // index of the live buffer per representation
    int count = 0;

    FrontierState(Ctx &cc, Workspace &w, int nn, long long cap) : c(cc), ws(w), n(nn), qcap(cap) {
        const size_t nb = ((size_t)nn + 255) / 256 * 256;
        ws.q[0].ensure((size_t)cap);
        ws.q[1].ensure((size_t)cap);
        ws.counters.ensure(64);
        ws.boolmap[0].ensure(nb);
        ws.boolmap[1].ensure(nb);
        ws.bitmap[0].ensure(nb / 64);
        ws.bitmap[1].ensure(nb / 64);
        ws.h_i32.ensure(16);
        fill_i32(c, ws.counters.p, 64, 0);
    }
    size_t nbytes_bool() const { return ((size_t)n + 255) / 256 * 256; }
    size_t nwords() const { return ((size_t)n + 255) / 256 * 4; }
    int32_t *cnt(int k) { return ws.counters.p + k; }

    int32_t *queue() { return ws.q[qi].p; }

    // make the live frontier available as a sparse queue
    const int32_t *as_queue() {
        if (rep == kRepQueue) return ws.q[qi].p;
        fill_i32(c, cnt(1), 1, 0);
        if (rep == kRepBoolmap) boolmap_to_queue(c, ws.boolmap[bi].p, n, ws.q[qi].p, cnt(1));
        else bitmap_to_queue(c, ws.bitmap[ti].p, n, ws.q[qi].p, cnt(1));
        rep = kRepQueue;
        return ws.q[qi].p;
    }
    const uint8_t *as_boolmap() {
        if (rep == kRepBoolmap) return ws.boolmap[bi].p;
        if (rep == kRepQueue) {
            fill_u8(c, ws.boolmap[bi].p, (long long)nbytes_bool(), 0);
            queue_to_boolmap(c, ws.q[qi].p, count, ws.boolmap[bi].p);
        } else {
            bitmap_to_boolmap(c, ws.bitmap[ti].p, n, ws.boolmap[bi].p);
        }
        rep = kRepBoolmap;
        return ws.boolmap[bi].p;
    }
    const unsigned long long *as_bitmap() {
        if (rep == kRepBitmap) return ws.bitmap[ti].p;
        if (rep == kRepQueue) {
            fill_u64(c, ws.bitmap[ti].p, (long long)nwords(), 0);
            queue_to_bitmap(c, ws.q[qi].p, count, ws.bitmap[ti].p);
        } else {
            boolmap_to_bitmap(c, ws.boolmap[bi].p, n, ws.bitmap[ti].p);
        }
        rep = kRepBitmap;
        return ws.bitmap[ti].p;
    }

    // Output frontier for a push with the given creation/dedup mode. With
    // FUSED creation under STRICT (lb) the output count is zeroed by the degree
    // scan that precedes the push instead of a launch of its own.
    OutFrontier prep_out(int create, int dedup, int iter, int lb = -1) {
        OutFrontier o{};
        o.overflow = cnt(2);
        if (create == kCreateFused) {
            if (lb == GG_LB_STRICT) o.clear = cnt(0);
            else fill_i32(c, cnt(0), 1, 0);
            o.q = ws.q[qi ^ 1].p;
            o.count = cnt(0);
            o.cap = (int32_t)qcap;
        } else if (create == kCreateBoolmap) {
            fill_u8(c, ws.boolmap[bi ^ 1].p, (long long)nbytes_bool(), 0);
            o.boolmap = ws.boolmap[bi ^ 1].p;
        } else {
            fill_u64(c, ws.bitmap[ti ^ 1].p, (long long)nwords(), 0);
            o.bitmap = ws.bitmap[ti ^ 1].p;
        }
        if (dedup == kDedupMonotonic) {
            o.tags = ws.tags.p;
            o.iter = iter;
        } else if (dedup == kDedupBitmap) {
            ws.dedup_bits.ensure(nwords());
            fill_u64(c, ws.dedup_bits.p, (long long)nwords(), 0);
            o.dedup_bits = ws.dedup_bits.p;
        } else if (dedup == kDedupBoolmap) {
            ws.dedup_bytes.ensure(nbytes_bool() / 4);
            fill_i32(c, reinterpret_cast<int32_t *>(ws.dedup_bytes.p), (long long)nbytes_bool() / 4, 0);
            o.dedup_bytes = ws.dedup_bytes.p;
        }
        return o;
    }

    // After the traversal: flip to the output buffer and read back its size.
    void commit(int create) {
        if (create == kCreateFused) {
            qi ^= 1;
            rep = kRepQueue;
        } else if (create == kCreateBoolmap) {
            bi ^= 1;
            rep = kRepBoolmap;
            fill_i32(c, cnt(0), 1, 0);
            count_boolmap(c, ws.boolmap[bi].p, n, cnt(0));
        } else {
            ti ^= 1;
            rep = kRepBitmap;
            fill_i32(c, cnt(0), 1, 0);
            count_bitmap(c, ws.bitmap[ti].p, n, cnt(0));
        }
        GG_HIP(hipMemcpyAsync(ws.h_i32.p, ws.counters.p, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
        GG_HIP(hipStreamSynchronize(c.s));
        count = ws.h_i32.p[0];
        if (ws.h_i32.p[2] != 0 || (create == kCreateFused && count > qcap))
            throw Error(GG_ERR_OUT_OF_MEMORY,
                        "output frontier exceeded its queue capacity (enable deduplication)");
    }

    // After a pull that wrote its output itself into the given representation
    // (queue -> next queue buffer, dense -> next dense buffer) and counted it
    // into cnt(0).
    void commit_pull(int create) {
        if (create == kCreateFused) { qi ^= 1; rep = kRepQueue; }
        else if (create == kCreateBoolmap) { bi ^= 1; rep = kRepBoolmap; }
        else { ti ^= 1; rep = kRepBitmap; }
        GG_HIP(hipMemcpyAsync(ws.h_i32.p, ws.counters.p, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
        GG_HIP(hipStreamSynchronize(c.s));
        count = ws.h_i32.p[0];
        if (ws.h_i32.p[2] != 0) throw Error(GG_ERR_OUT_OF_MEMORY, "output frontier exceeded its capacity");
    }
};

// Pick the schedule of this iteration (HybridGPUSchedule, INPUT_VERTEXSET_SIZE).
inline const gg_simple_schedule &pick(const gg_schedule &s, long long count, int n) {
    if (s.hybrid && (double)count > (double)s.threshold * (double)n) return s.s2;
    return s.s1;
}

struct StatsScope {
    gg_stats *st;
    Ctx &c;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DevBuf<unsigned long long> ecount;
    StatsScope(gg_stats *s, Ctx &cc) : st(s), c(cc) {
        if (!st) return;
        const uint32_t flags = st->flags;
        *st = gg_stats{};
        st->flags = flags;
        if (flags & GG_STATS_COUNT_EDGES) {
            ecount.ensure(1);
            fill_u64(c, ecount.p, 1, 0ull);
            c.edge_counter = ecount.p;
        }
        GG_HIP(hipEventCreate(&e0));
        GG_HIP(hipEventCreate(&e1));
        GG_HIP(hipEventRecord(e0, c.s));
    }
    void finish() {
        if (!st) return;
        GG_HIP(hipEventRecord(e1, c.s));
        GG_HIP(hipEventSynchronize(e1));
        float ms = 0;
        GG_HIP(hipEventElapsedTime(&ms, e0, e1));
        st->device_ms = ms;
        st->launches = c.launches;
        if (c.edge_counter) {
            unsigned long long v = 0;
            GG_HIP(hipMemcpy(&v, c.edge_counter, sizeof(v), hipMemcpyDeviceToHost));
            st->edges_examined = (int64_t)v;
        }
    }
    ~StatsScope() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace gg
