// Frontier representations and output-frontier creation.
//
// Representations (GPU Optimization Space section, "Active Vertexset
// Creation"; SimpleGPUSchedule table, configDirection/configFrontierCreation):
//   sparse queue : int32 ids[cap] + int32 count
//   boolmap      : uint8 per vertex (no atomics needed to set)
//   bitmap       : one bit per vertex in uint64 words (wave64 ballot writes a
//                  whole word; scattered sets need an atomic OR)
// Deduplication (configDeduplication; "Active Vertexset Deduplication"):
//   monotonic counters : tag[v] raised to the iteration id by an atomic max;
//                        the raising call enqueues, the tags are never cleared
//   bitmap / boolmap   : test-and-set of v's bit / byte, cleared every round
#pragma once

#include "common.hpp"

namespace gg {

enum CreateMode : int { kCreateFused = 0, kCreateBoolmap = 1, kCreateBitmap = 2 };
enum DedupMode : int { kDedupNone = 0, kDedupMonotonic = 1, kDedupBitmap = 2, kDedupBoolmap = 3 };

struct OutFrontier {
    int32_t *q;              // FUSED: output queue
    int32_t *count;          // FUSED: output count (device)
    int32_t cap;             // FUSED: queue capacity
    int32_t *overflow;       // set to 1 when an enqueue would pass `cap`
    uint8_t *boolmap;        // UNFUSED_BOOLMAP output
    unsigned long long *bitmap;  // UNFUSED_BITMAP output
    int32_t *tags;           // MONOTONIC_COUNTERS
    int32_t iter;            // MONOTONIC_COUNTERS: id of this iteration (>= 1)
    unsigned long long *dedup_bits;  // BITMAP dedup (cleared every round)
    unsigned *dedup_bytes;   // BOOLMAP dedup, bytes packed 4 per word (cleared every round)
    int32_t *clear;          // FUSED: `count` when its creator left zeroing it to the traversal's
                             // first kernel (STRICT's degree scan), else null
};

// Each test reads the tag first and skips the atomic when v is already
// marked (tags and bits only grow within a round; a stale read only costs the
// atomic), which keeps repeated enqueues of popular vertices off one address.
template <int DEDUP>
__device__ __forceinline__ bool dedup_first(const OutFrontier &o, int v) {
    if constexpr (DEDUP == kDedupMonotonic) {
        if (o.tags[v] >= o.iter) return false;
        return atomic_max_i32(&o.tags[v], o.iter) < o.iter;
    } else if constexpr (DEDUP == kDedupBitmap) {
        const unsigned long long bit = 1ull << (v & 63);
        if (o.dedup_bits[v >> 6] & bit) return false;
        return (atomic_or_u64(&o.dedup_bits[v >> 6], bit) & bit) == 0;
    } else if constexpr (DEDUP == kDedupBoolmap) {
        const unsigned sh = (unsigned)(v & 3) * 8u;
        if ((o.dedup_bytes[v >> 2] >> sh) & 1u) return false;
        return ((atomic_or_u32(&o.dedup_bytes[v >> 2], 1u << sh) >> sh) & 1u) == 0;
    } else {
        return true;
    }
}

// dedup_first over a lane's batch of B candidates (want[b] in: x[b] is a
// candidate; out: x[b] is its first enqueue this round). All tag reads are
// issued, then all atomics, then the results are read: each atomic's result
// starts out as the value read (a value the compiler cannot fold), so the
// result test is not moved into the atomic's branch, where it would make the
// lane wait for every atomic in turn.
template <int DEDUP, int B>
__device__ __forceinline__ void dedup_batch(const OutFrontier &o, const int *x, bool *want) {
    if constexpr (DEDUP == kDedupMonotonic) {
        int r[B];
#pragma unroll
        for (int b = 0; b < B; b++) r[b] = want[b] ? o.tags[x[b]] : o.iter;
#pragma unroll
        for (int b = 0; b < B; b++)
            if (want[b] && r[b] < o.iter) r[b] = atomic_max_i32(&o.tags[x[b]], o.iter);
#pragma unroll
        for (int b = 0; b < B; b++) want[b] = want[b] && r[b] < o.iter;
    } else if constexpr (DEDUP == kDedupBitmap) {
        unsigned long long r[B];
#pragma unroll
        for (int b = 0; b < B; b++) r[b] = want[b] ? o.dedup_bits[x[b] >> 6] : ~0ull;
#pragma unroll
        for (int b = 0; b < B; b++) {
            const unsigned long long bit = 1ull << (x[b] & 63);
            if (want[b] && !(r[b] & bit)) r[b] = atomic_or_u64(&o.dedup_bits[x[b] >> 6], bit);
        }
#pragma unroll
        for (int b = 0; b < B; b++) want[b] = want[b] && !((r[b] >> (x[b] & 63)) & 1ull);
    } else if constexpr (DEDUP == kDedupBoolmap) {
        unsigned r[B];
#pragma unroll
        for (int b = 0; b < B; b++) r[b] = want[b] ? o.dedup_bytes[x[b] >> 2] : ~0u;
#pragma unroll
        for (int b = 0; b < B; b++) {
            const unsigned sh = (unsigned)(x[b] & 3) * 8u;
            if (want[b] && !((r[b] >> sh) & 1u)) r[b] = atomic_or_u32(&o.dedup_bytes[x[b] >> 2], 1u << sh);
        }
#pragma unroll
        for (int b = 0; b < B; b++) want[b] = want[b] && !((r[b] >> ((unsigned)(x[b] & 3) * 8u)) & 1u);
    }
}

// Wave-aggregated append: one atomic per wavefront, lanes write at
// base + (number of wanting lanes below them). Every active lane of the
// wave must call this together.
__device__ __forceinline__ void wave_append(int32_t *q, int32_t *count, int32_t cap, int32_t *overflow,
                                            bool want, int v) {
    const uint64_t mask = __ballot(want);
    if (mask == 0) return;
    const int leader = first_lane(mask);
    int base = 0;
    if (lane_id() == leader) base = atomic_add_i32(count, __popcll(mask));
    base = wave_bcast(base, leader);
    if (want) {
        const int pos = base + lanes_below(mask);
        if (pos < cap) q[pos] = v;
        else *overflow = 1;
    }
}

// Appends staged per workgroup: lanes reserve LDS slots (one LDS atomic per
// wavefront) and the workgroup publishes them with one global atomic when it
// flushes. Every workgroup of a traversal appends to the same queue, so
// per-wavefront global atomics serialise on one address (measured: halving
// the batched SSSP loop's time); slots past the LDS capacity fall back to
// the per-wavefront global append.
constexpr int kStage = 2048;

struct Staged {
    int32_t *sq;     // LDS slots
    int *sc;         // LDS count (may pass kStage: the excess went global)
    int32_t *q;      // global queue
    int32_t *count;  // its global count
};

__device__ __forceinline__ void stage_append(const Staged &st, int32_t cap, int32_t *overflow, bool want, int v) {
    const uint64_t mask = __ballot(want);
    if (mask == 0) return;
    const int leader = first_lane(mask);
    int base = 0;
    if (lane_id() == leader) base = __hip_atomic_fetch_add(st.sc, __popcll(mask), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
    base = wave_bcast(base, leader);
    const int pos = base + lanes_below(mask);
    if (want && pos < kStage) st.sq[pos] = v;
    wave_append(st.q, st.count, cap, overflow, want && pos >= kStage, v);
}

// every lane of the workgroup calls this; leaves the LDS count at zero
__device__ __forceinline__ void stage_flush(const Staged &st, int32_t cap, int32_t *overflow, int *s_base) {
    __syncthreads();
    const int cnt = min(*st.sc, kStage);
    if (threadIdx.x == 0) *s_base = cnt > 0 ? atomic_add_i32(st.count, cnt) : 0;
    __syncthreads();
    const int base = *s_base;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        if (base + i < cap) st.q[base + i] = st.sq[i];
        else *overflow = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) *st.sc = 0;
    __syncthreads();
}

// B appends per lane at once (lane l wants v[b] when want[b]). Every lane of
// the wavefront must call this together: the lanes' counts are placed with one
// scan and one LDS atomic per wavefront, and the slots past the stage with one
// global atomic. st.sq must have kStage + 1 slots (StageLDS's do).
template <int B>
__device__ __forceinline__ void stage_append_batch(const Staged &st, int32_t cap, int32_t *overflow, const int *v,
                                                   const bool *want) {
    int k = 0;
#pragma unroll
    for (int b = 0; b < B; b++) k += want[b];
    const int incl = wave_incl_scan(k);
    const int total = wave_bcast(incl, kWave - 1);
    if (total == 0) return;
    int base = 0;
    if (lane_id() == kWave - 1)
        base = __hip_atomic_fetch_add(st.sc, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    base = wave_bcast(base, kWave - 1);
    // slots [lo, base + total) lie past the stage: one global reservation for
    // all of them (a hub's walk can fill the stage long before a flush)
    const int lo = base > kStage ? base : kStage;
    const int n_over = base + total - lo;
    int gbase = 0;
    if (n_over > 0) {
        if (lane_id() == kWave - 1) gbase = atomic_add_i32(st.count, n_over);
        gbase = wave_bcast(gbase, kWave - 1);
    }
    int pos = base + incl - k;
    if (n_over <= 0) {
        // all of the wavefront's slots are in the stage: unwanted items write
        // the sink slot sq[kStage], so no item needs a branch
#pragma unroll
        for (int b = 0; b < B; b++) {
            st.sq[want[b] ? pos : kStage] = v[b];
            pos += want[b];
        }
        return;
    }
#pragma unroll
    for (int b = 0; b < B; b++) {
        if (want[b]) {
            if (pos < kStage) {
                st.sq[pos] = v[b];
            } else {
                const int q = gbase + (pos - lo);
                if (q < cap) st.q[q] = v[b];
                else *overflow = 1;
            }
        }
        pos += want[b];
    }
}

// Output-frontier sink used inside edge loops (FUSED creation calls the
// wave-aggregated append; the unfused forms mark a dense map).
template <int CREATE, int DEDUP>
__device__ __forceinline__ void emit(const OutFrontier &o, bool want, int v) {
    if constexpr (CREATE == kCreateFused) {
        if (want) want = dedup_first<DEDUP>(o, v);
        wave_append(o.q, o.count, o.cap, o.overflow, want, v);
    } else if constexpr (CREATE == kCreateBoolmap) {
        if (want) o.boolmap[v] = 1;
    } else {
        if (want) atomic_or_u64(&o.bitmap[v >> 6], 1ull << (v & 63));
    }
}

// Workgroup-staged form of emit (FUSED creation stages in LDS; the dense-map
// forms need no queue). `s` is the workgroup's LDS stage; the caller flushes
// it at workgroup-uniform points.
struct StageLDS {
    int32_t q[kStage + 1];  // the last slot takes the batch appends' discarded writes
    int c, base;
};

template <int CREATE, int DEDUP>
__device__ __forceinline__ void emit_staged(const OutFrontier &o, StageLDS &s, bool want, int v) {
    if constexpr (CREATE == kCreateFused) {
        if (want) want = dedup_first<DEDUP>(o, v);
        stage_append(Staged{s.q, &s.c, o.q, o.count}, o.cap, o.overflow, want, v);
    } else {
        emit<CREATE, DEDUP>(o, want, v);
    }
}

// emit_staged for a lane's batch of B results (x[b] >= 0: append x[b]); every
// lane of the wavefront calls it together
template <int CREATE, int DEDUP, int B>
__device__ __forceinline__ void emit_staged_batch(const OutFrontier &o, StageLDS &s, const int *x) {
    if constexpr (CREATE == kCreateFused) {
        bool want[B];
#pragma unroll
        for (int b = 0; b < B; b++) want[b] = x[b] >= 0;
        dedup_batch<DEDUP, B>(o, x, want);
        stage_append_batch<B>(Staged{s.q, &s.c, o.q, o.count}, o.cap, o.overflow, x, want);
    } else {
#pragma unroll
        for (int b = 0; b < B; b++) emit<CREATE, DEDUP>(o, x[b] >= 0, x[b]);
    }
}

template <int CREATE>
__device__ __forceinline__ void emit_flush(const OutFrontier &o, StageLDS &s) {
    if constexpr (CREATE == kCreateFused) stage_flush(Staged{s.q, &s.c, o.q, o.count}, o.cap, o.overflow, &s.base);
}

// Flush only once the stage is at least half full. Every flush is an atomic
// on the one queue count shared by the whole grid, and atomics on one
// address serialise (~11 ns each here): flushing every workgroup iteration
// made tens of thousands of them per launch. Appends past a full stage fall
// back to per-wavefront appends; the caller flushes the rest after its loop.
// Every lane of the workgroup calls this.
template <int CREATE>
__device__ __forceinline__ void emit_flush_half(const OutFrontier &o, StageLDS &s) {
    if constexpr (CREATE == kCreateFused) {
        __syncthreads();
        const bool go = s.c >= kStage / 2;
        __syncthreads();
        if (go) stage_flush(Staged{s.q, &s.c, o.q, o.count}, o.cap, o.overflow, &s.base);
    }
}

// ---- dense-map membership ----------------------------------------------------------
__device__ __forceinline__ bool bit_test(const unsigned long long *bm, int v) {
    return (bm[v >> 6] >> (v & 63)) & 1ull;
}

// ---- sources of an edge traversal ---------------------------------------------------
struct SrcQueue {  // explicit frontier
    const int32_t *ids;
    int32_t size;
    __device__ __forceinline__ int get(int i) const { return ids[i]; }
};
struct SrcAll {  // every vertex (topology-driven and pull traversals)
    int32_t size;
    __device__ __forceinline__ int get(int i) const { return i; }
};

}  // namespace gg
