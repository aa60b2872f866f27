// Shared device/host helpers for the gfx950 traversal kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/gg.h"

namespace gg {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kBlock = 256;     // default workgroup size (4 wavefronts)

// ---- errors ------------------------------------------------------------------
struct Error : std::runtime_error {
    gg_status code;
    Error(gg_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define GG_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)           \
                throw ::gg::Error(GG_ERR_OUT_OF_MEMORY,                                \
                                  std::string(#call) + ": " + hipGetErrorString(e_));  \
            throw ::gg::Error(GG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

#define GG_CHECK_LAUNCH() GG_HIP(hipGetLastError())

inline void require(bool ok, gg_status code, const std::string &msg) {
    if (!ok) throw Error(code, msg);
}

// ---- device-side graph view -----------------------------------------------------
struct DevGraph {
    int32_t n;
    int64_t m;
    const int32_t *__restrict__ row_ptr;  // [n+1]
    const int32_t *__restrict__ col;      // [m]
    const uint32_t *__restrict__ w;       // [m] or null
    const int32_t *__restrict__ coo_src;  // [m] source of each CSR entry (EDGE_ONLY) or null
    // in-edges for PULL: the CSR itself on a symmetric graph, else its
    // transpose (in-rows sorted by source; null until built)
    const int32_t *__restrict__ in_row_ptr;
    const int32_t *__restrict__ in_col;
};

// ---- wavefront helpers -----------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// number of set bits of `mask` strictly below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int first_lane(uint64_t mask) { return __ffsll((unsigned long long)mask) - 1; }

template <class T>
__device__ __forceinline__ T wave_bcast(T v, int src_lane) { return __shfl(v, src_lane, kWave); }

// inclusive prefix sum over the 64 lanes (all lanes must be active)
__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ long long wave_incl_scan64(long long x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        long long y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// ---- atomics (agent scope: visible across all XCDs) ---------------------------------
__device__ __forceinline__ int atomic_add_i32(int *p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_add_u64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_min_i32(int *p, int v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_max_i32(int *p, int v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_cas_i32(int *p, int expected, int desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expected;  // old value
}
__device__ __forceinline__ unsigned atomic_or_u32(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_or_u64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float atomic_add_f32(float *p, float v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double atomic_add_f64(double *p, double v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- launch helpers ---------------------------------------------------------------
inline unsigned blocks_for(long long work, int per_block, unsigned cap = 1u << 20) {
    long long b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (long long)cap) b = cap;
    return (unsigned)b;
}

}  // namespace gg
