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
    int32_t q[kStage];
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
