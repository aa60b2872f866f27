// Shared pieces of the single- and multi-source Brandes passes: the
// dependency accumulation step and the degree tiers that fix the order of
// every vertex's sum (identical in both, so their results agree bit for bit).
#pragma once

#include "common.hpp"

namespace gg {

constexpr int kBcWaveDeg = 64, kBcBlockDeg = 4096;

// Brandes' dependency delta(v) = sum over successors w of sigma(v)/sigma(w) *
// (1 + delta(w)) is evaluated as sigma(v) * sum_w t(w) with
// t(w) = (1 + delta(w)) / sigma(w): each vertex stores t once its delta is
// final, and a predecessor gathers one value per successor edge instead of
// sigma(w) and delta(w). No contraction into FMA, so every kernel rounds the
// same way.
__device__ __forceinline__ double bc_tval(double sw, double dw) {
#pragma clang fp contract(off)
    return (1.0 + dw) / sw;
}
__device__ __forceinline__ double bc_delta(double sv, double sum_t) {
#pragma clang fp contract(off)
    return sv * sum_t;
}

}  // namespace gg
