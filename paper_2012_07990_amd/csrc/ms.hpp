// Shared pieces of the batched multi-source kernels: per-source state is
// kept vertex-major (the K values of a vertex are adjacent, so the sources
// relaxing one edge touch one cache line) and transposed into k x n row-major
// outputs at the end.
#pragma once

#include "common.hpp"

namespace gg {

// ---- vertex-major (n x K) -> row-major (rows j0.. of a k x n output), tiled through LDS
template <class TI, class TO>
__global__ __launch_bounds__(kBlock) void k_ms_transpose(const TI *in, int n, int K, TO *out, int j0) {
    __shared__ TI tile[64][65];
    for (int v0 = blockIdx.x * 64; v0 < n; v0 += gridDim.x * 64) {
        for (int i = threadIdx.x; i < 64 * K; i += kBlock) {
            const int dv = i / K, j = i % K;
            if (v0 + dv < n) tile[j][dv] = in[(size_t)(v0 + dv) * K + j];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * K; i += kBlock) {
            const int j = i / 64, dv = i % 64;
            if (v0 + dv < n) out[(size_t)(j0 + j) * n + v0 + dv] = (TO)tile[j][dv];
        }
        __syncthreads();
    }
}

}  // namespace gg
