// Shared pieces of the single- and multi-source Brandes passes: the
// dependency accumulation step and the degree tiers that fix the order of
// every vertex's sum (identical in both, so their results agree bit for bit).
#pragma once

#include "common.hpp"

namespace gg {

constexpr int kBcWaveDeg = 64, kBcBlockDeg = 4096;

// acc + sigma(v)/sigma(w) * (1 + delta(w)) with no contraction into FMA, so
// every kernel rounds this expression the same way
__device__ __forceinline__ double bc_step(double acc, double sv, double sw, double dw) {
#pragma clang fp contract(off)
    const double q = sv / sw;
    const double t = q * (1.0 + dw);
    return acc + t;
}

}  // namespace gg
