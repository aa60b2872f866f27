// Generic push edgeset.apply: launches the load-balancing strategy chosen by
// the schedule over a sparse input frontier, with the chosen output-frontier
// creation and deduplication (SimpleGPUSchedule table). Included by each
// algorithm's translation unit, which instantiates it with its edge functor.
#pragma once

#include "lb.hpp"
#include "ops.hpp"

namespace gg {

template <int LB, int CREATE, int DEDUP, class F>
__global__ __launch_bounds__(kBlock) void k_push(DevGraph g, SrcQueue src, F f, OutFrontier out,
                                                 const long long *scan, const uint8_t *member,
                                                 unsigned long long *ecount) {
    long long ne = 0;
    const Tid t = Tid::here();
    if constexpr (LB == GG_LB_VERTEX_BASED) lb_vp<CREATE, DEDUP>(g, src, f, out, t, ne);
    else if constexpr (LB == GG_LB_WM) lb_wm<CREATE, DEDUP>(g, src, f, out, t, ne);
    else if constexpr (LB == GG_LB_CM) lb_cm<CREATE, DEDUP>(g, src, f, out, t, ne);
    else if constexpr (LB == GG_LB_ETWC) lb_etwc<CREATE, DEDUP>(g, src, f, out, t, ne);
    else if constexpr (LB == GG_LB_STRICT) lb_strict<CREATE, DEDUP>(g, src, scan, f, out, t, ne);
    else if constexpr (LB == GG_LB_EDGE_ONLY) lb_edge_only<CREATE, DEDUP>(g, member, f, out, t, ne);
    flush_edge_count(ne, ecount);
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_twc_bin(DevGraph g, SrcQueue src, F f, TwcBins b) {
    twc_bin(g, src, f, b, Tid::here());
}

template <int CREATE, int DEDUP, class F>
__global__ __launch_bounds__(kBlock) void k_twc_tier(int tier, DevGraph g, const int32_t *ids,
                                                     const int32_t *size_ptr, F f, OutFrontier out,
                                                     unsigned long long *ecount) {
    long long ne = 0;
    const Tid t = Tid::here();
    const int size = *size_ptr;
    if (tier == 0) lb_vp<CREATE, DEDUP>(g, SrcQueue{ids, size}, f, out, t, ne);
    else if (tier == 1) twc_wave_tier<CREATE, DEDUP>(g, ids, size, f, out, t, ne);
    else twc_block_tier<CREATE, DEDUP>(g, ids, size, f, out, t, ne);
    flush_edge_count(ne, ecount);
}

// Build the COO source array once per graph (EDGE_ONLY needs it).
void ensure_coo(Ctx &c, Graph &G);

struct PushPlan {
    int lb, create, dedup;  // dedup is a DedupMode
};

template <int LB, int CREATE, int DEDUP, class F>
static void launch_push_lb(Ctx &c, const DevGraph &g, Workspace &ws, const int32_t *q, int qn, F &f,
                           const OutFrontier &out, uint8_t *member_scratch) {
    const unsigned cap = 65535;
    if constexpr (LB == GG_LB_TWC) {
        ws.bins.ensure((size_t)3 * (size_t)(qn > 0 ? qn : 1));
        int32_t *cnt = ws.counters.p + 8;
        fill_i32(c, cnt, 3, 0);
        TwcBins b{{ws.bins.p, ws.bins.p + qn, ws.bins.p + 2 * (size_t)qn}, cnt, qn, out.overflow};
        hipLaunchKernelGGL(k_twc_bin<F>, dim3(blocks_for(qn, kBlock, cap)), dim3(kBlock), 0, c.s, g,
                           SrcQueue{q, qn}, f, b);
        GG_CHECK_LAUNCH();
        hipLaunchKernelGGL((k_twc_tier<CREATE, DEDUP, F>), dim3(blocks_for(qn, kBlock, cap)), dim3(kBlock), 0,
                           c.s, 0, g, b.q[0], cnt + 0, f, out, c.edge_counter);
        GG_CHECK_LAUNCH();
        hipLaunchKernelGGL((k_twc_tier<CREATE, DEDUP, F>), dim3(blocks_for(qn, kBlock / kWave, cap)),
                           dim3(kBlock), 0, c.s, 1, g, b.q[1], cnt + 1, f, out, c.edge_counter);
        GG_CHECK_LAUNCH();
        hipLaunchKernelGGL((k_twc_tier<CREATE, DEDUP, F>), dim3(blocks_for(qn, 1, 8192)), dim3(kBlock), 0,
                           c.s, 2, g, b.q[2], cnt + 2, f, out, c.edge_counter);
        GG_CHECK_LAUNCH();
        c.launches += 5;
        return;
    } else {
        const long long *scan = nullptr;
        unsigned blocks = blocks_for(qn, kBlock, cap);
        if constexpr (LB == GG_LB_STRICT) {
            ws.scan.ensure((size_t)qn + 1);
            ws.scan_part.ensure(degree_scan_partials(qn));
            degree_scan(c, g, q, qn, ws.scan.p, ws.scan_part.p, out.clear);
            scan = ws.scan.p;
            blocks = (unsigned)c.num_cus * 8;
        }
        if constexpr (LB == GG_LB_EDGE_ONLY) {
            require(g.coo_src != nullptr && member_scratch != nullptr, GG_ERR_DEVICE,
                    "EDGE_ONLY needs the COO source array and a membership map");
            fill_u8(c, member_scratch, ((long long)g.n + 255) / 256 * 256, 0);
            queue_to_boolmap(c, q, qn, member_scratch);
            blocks = blocks_for(g.m, kBlock, 16384);
        }
        hipLaunchKernelGGL((k_push<LB, CREATE, DEDUP, F>), dim3(blocks), dim3(kBlock), 0, c.s, g,
                           SrcQueue{q, qn}, f, out, scan, (const uint8_t *)member_scratch, c.edge_counter);
        GG_CHECK_LAUNCH();
        c.launches++;
    }
}

template <int CREATE, int DEDUP, class F>
static void launch_push_cd(Ctx &c, const DevGraph &g, Workspace &ws, int lb, const int32_t *q, int qn, F &f,
                           const OutFrontier &out, uint8_t *member) {
    switch (lb) {
    case GG_LB_VERTEX_BASED: launch_push_lb<GG_LB_VERTEX_BASED, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_WM: launch_push_lb<GG_LB_WM, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_CM: launch_push_lb<GG_LB_CM, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_STRICT: launch_push_lb<GG_LB_STRICT, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_TWC: launch_push_lb<GG_LB_TWC, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_ETWC: launch_push_lb<GG_LB_ETWC, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    case GG_LB_EDGE_ONLY: launch_push_lb<GG_LB_EDGE_ONLY, CREATE, DEDUP>(c, g, ws, q, qn, f, out, member); break;
    default: throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, "unknown load-balance mode");
    }
}

// One push edgeset.apply over q[0..qn). `member` is an n-byte scratch map
// (EDGE_ONLY only). Output and dedup buffers in `out` must be prepared.
template <class F>
void push_apply(Ctx &c, const DevGraph &g, Workspace &ws, const PushPlan &p, const int32_t *q, int qn, F f,
                const OutFrontier &out, uint8_t *member) {
    if (qn <= 0) {
        if (out.clear) fill_i32(c, out.clear, 1, 0);
        return;
    }
    if (p.create == kCreateFused) {
        switch (p.dedup) {
        case kDedupNone: launch_push_cd<kCreateFused, kDedupNone>(c, g, ws, p.lb, q, qn, f, out, member); break;
        case kDedupMonotonic: launch_push_cd<kCreateFused, kDedupMonotonic>(c, g, ws, p.lb, q, qn, f, out, member); break;
        case kDedupBitmap: launch_push_cd<kCreateFused, kDedupBitmap>(c, g, ws, p.lb, q, qn, f, out, member); break;
        case kDedupBoolmap: launch_push_cd<kCreateFused, kDedupBoolmap>(c, g, ws, p.lb, q, qn, f, out, member); break;
        default: throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, "unknown dedup mode");
        }
    } else if (p.create == kCreateBoolmap) {
        launch_push_cd<kCreateBoolmap, kDedupNone>(c, g, ws, p.lb, q, qn, f, out, member);
    } else {
        launch_push_cd<kCreateBitmap, kDedupNone>(c, g, ws, p.lb, q, qn, f, out, member);
    }
}

// n-byte scratch map for EDGE_ONLY's input-frontier membership
inline uint8_t *member_map(Workspace &ws, int n, int lb) {
    if (lb != GG_LB_EDGE_ONLY) return nullptr;
    ws.member.ensure(((size_t)n + 255) / 256 * 256);
    return ws.member.p;
}

// Map a schedule's dedup fields to a DedupMode (only FUSED creation dedups:
// the dense maps are duplicate-free by construction).
inline int dedup_mode(const gg_simple_schedule &s) {
    if (s.frontier_creation != GG_CREATE_FUSED || !s.dedup_enable) return kDedupNone;
    switch (s.dedup_type) {
    case GG_DEDUP_MONOTONIC_COUNTERS: return kDedupMonotonic;
    case GG_DEDUP_BITMAP: return kDedupBitmap;
    case GG_DEDUP_BOOLMAP: return kDedupBoolmap;
    default: return kDedupMonotonic;
    }
}

}  // namespace gg
