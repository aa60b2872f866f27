"""Benchmark: GTEPS of the five traversal algorithms on a synthetic R-MAT
scale-22 graph (4,194,304 vertices, edge factor 16, a/b/c/d = .57/.19/.19/.05,
symmetrised, self-loops and duplicates removed) on one MI355X.

One step = one pass of the whole hot path over the resident graph:
direction-optimising BFS, delta-stepping SSSP, CC (hooking + shortcutting),
PageRank (FP32, 20 rounds, d = 0.85) and single-source BC, each under its
tuned schedule. `value` is the aggregate GTEPS of the step: traversed edges
(BFS/SSSP/BC: sum of degrees of reached vertices; CC: m; PR: 20 m) over the
step's wall time with the graph already in HBM.

Prints ONE JSON line (rank 0). `--gpus N` with N > 1 is refused: the library
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _report_exit():
    print("bench: library objects closed, interpreter exiting", file=sys.stderr, flush=True)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s
PR_SEGMENT = 1 << 20   # PageRank pull EdgeBlocking: source segments of 2^20 vertices
PR_LDS_SOURCES = 12288 # highest-degree sources per segment the STRICT kernel keeps in LDS
CC_SEGMENT = 1 << 20   # CC hook sweep: pairs blocked by destination segments of 2^20 vertices
SSSP_SEGMENT = 1 << 21 # SSSP dense rounds: EdgeBlocked COO with destination segments of 2^21 vertices
SSSP_DENSE = 0.2       # SSSP rounds whose frontier holds more than this share of the vertices are dense


def measured_traffic(kernel_src: str, summary: str, schedule_tag: str):
    """HBM bytes per launch from a committed rocprofv3 summary, when that
    summary was taken on the current kernel source under the same schedule
    (else None)."""
    import hashlib
    import re
    try:
        h = hashlib.sha256(open(os.path.join(ROOT, kernel_src), "rb").read()).hexdigest()[:16]
        txt = open(os.path.join(ROOT, "profiles", summary)).read()
    except OSError:
        return None
    if h not in txt or ("schedule: %s" % schedule_tag) not in txt:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--only", default="", help="comma list of algorithms to run (bfs,sssp,cc,pr,bc)")
    p.add_argument("--sweep", action="store_true", help="time every schedule family per algorithm")
    p.add_argument("--sweep-filter", default="",
                   help="comma list of substrings of 'algo/schedule': only sweep schedules matching one")
    p.add_argument("--counters-sweep", action="store_true",
                   help="for rocprofv3 --pmc runs: run each (filtered) sweep schedule twice after a warm run, "
                        "bracketed by marker launches (a one-element torch.cumsum before and after), print "
                        "the schedule order and exit")
    p.add_argument("--verbose", action="store_true")
    p.add_argument("--no-batched", action="store_true", help="skip the batched multi-source section")
    p.add_argument("--no-serving", action="store_true", help="skip the serving section")
    p.add_argument("--serve-rates", default="100,500,1000,2000,5000", help="Poisson arrival rates (queries/s)")
    p.add_argument("--serve-seconds", type=float, default=5.0, help="seconds of arrivals per rate")
    p.add_argument("--serve-baseline-s", type=float, default=5.0,
                   help="wall-clock cap of the one-query-per-launch baseline at each rate")
    p.add_argument("--serve-budget-s", type=float, default=150.0, help="wall-clock cap of the serving section")
    p.add_argument("--grid", type=int, default=4096,
                   help="side of the road-like grid for the BFS/SSSP fused-vs-unfused and delta runs (0: skip)")
    p.add_argument("--grid-deltas", default="1,8,64,512", help="delta values of the grid SSSP runs")
    p.add_argument("--grid-unfused-cap-s", type=float, default=4.0,
                   help="skip the unfused run of a grid configuration whose fused run took longer than this")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the autotuner section (per algorithm on R-MAT 22, its picks beside the step's schedules)")
    p.add_argument("--tune-budget-s", type=float, default=8.0, help="autotuner wall-clock budget per algorithm")
    p.add_argument("--pr-segment", type=int, default=PR_SEGMENT,
                   help="PageRank pull EdgeBlocking segment width (source vertices per segment)")
    p.add_argument("--no-placement", action="store_true",
                   help="skip the CPU-backend / placement section (SSSP and BFS on the 2048^2 grid and R-MAT 20)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy three times (scales rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def schedules(gg, pr_segment=PR_SEGMENT):
    """The schedule each algorithm runs in the step (chosen by sweeps on this graph family)."""
    bfs = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    bfs.s1.load_balance = gg.LB_STRICT
    bfs.threshold = 0.01
    sssp = gg.make_schedule(lb="strict", delta=4096, threshold=SSSP_DENSE,
                            hybrid={"lb": "edge_only", "edge_blocking": 1, "blocking_size": SSSP_SEGMENT,
                                    "frontier_creation": gg.CREATE_UNFUSED_BOOLMAP})
    cc = gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=CC_SEGMENT)
    pr = gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=pr_segment)
    bc = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
    bc.s1.load_balance = gg.LB_STRICT
    bc.threshold = 0.01
    return {"bfs": bfs, "sssp": sssp, "cc": cc, "pr": pr, "bc": bc}


def sweep_schedules(gg):
    out = {"bfs": {}, "sssp": {}, "cc": {}, "pr": {}, "bc": {}}
    for lb in ["vp", "wm", "cm", "strict", "twc", "etwc"]:
        out["bfs"]["push-" + lb] = gg.make_schedule(lb=lb)
        out["cc"][lb] = gg.make_schedule(lb=lb)
        out["cc"]["fused-" + lb] = gg.make_schedule(lb=lb, fusion=True)
    for th in [0.005, 0.01, 0.02]:
        for lb in ["strict", "twc", "cm"]:
            s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
            s.s1.load_balance = gg.LB_NAMES[lb]
            s.threshold = th
            out["bfs"]["hybrid-%s-%g" % (lb, th)] = s
    out["cc"]["edge_only"] = gg.make_schedule(lb="edge_only")
    for N in [1 << 18, 1 << 19, 1 << 20, 1 << 21]:
        out["cc"]["edge_only-eb-%d" % N] = gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=N)
    for th in [0.001, 0.01, 0.05, 0.2]:
        s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_BFS_HYBRID)
        s.threshold = th
        out["bfs"]["hybrid-vp-%g" % th] = s
        s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
        s.threshold = th
        out["bfs"]["hybrid-etwc-%g" % th] = s
    out["bfs"]["fused-vp"] = gg.make_schedule(lb="vp", fusion=True)
    for lb in ["vp", "strict"]:
        for th in [0.001, 0.01]:
            out["bfs"]["fused-hybrid-%s-%g" % (lb, th)] = gg.make_schedule(
                lb=lb, fusion=True, threshold=th, hybrid={"direction": gg.PULL, "pull_rep": gg.REP_BITMAP, "lb": "vp"})
    for d in [16, 64, 256, 1024]:
        for lb in ["wm", "etwc", "cm", "strict", "twc"]:
            out["sssp"]["%s-d%d" % (lb, d)] = gg.make_schedule(lb=lb, delta=d)
        out["sssp"]["fused-etwc-d%d" % d] = gg.make_schedule(lb="etwc", delta=d, fusion=True)
    for d in [2048, 4096, 16384, 1 << 20]:
        out["sssp"]["strict-d%d" % d] = gg.make_schedule(lb="strict", delta=d)
        out["sssp"]["fused-strict-d%d" % d] = gg.make_schedule(lb="strict", delta=d, fusion=True)
    out["cc"]["fused-strict"] = gg.make_schedule(lb="strict", fusion=True)
    for th in [0.01, 0.05, 0.1, 0.2, 0.3]:
        for N in [1 << 18, 1 << 19, 1 << 20, 1 << 21]:
            for cr, tag in [(gg.CREATE_FUSED, "q"), (gg.CREATE_UNFUSED_BOOLMAP, "bool")]:
                out["sssp"]["hybrid-strict-eb%d-%s-%g" % (N, tag, th)] = gg.make_schedule(
                    lb="strict", delta=4096, threshold=th,
                    hybrid={"lb": "edge_only", "edge_blocking": 1, "blocking_size": N, "frontier_creation": cr})
    out["sssp"]["strict-d64-nodedup"] = gg.make_schedule(lb="strict", delta=64, dedup=False)
    out["sssp"]["strict-d64-bitmapdedup"] = gg.make_schedule(lb="strict", delta=64, dedup_type=gg.DEDUP_BITMAP)
    for lb in ["vp", "wm", "etwc", "strict"]:
        out["pr"]["pull-" + lb] = gg.make_schedule(lb=lb, direction=gg.PULL)
    out["pr"]["push-edge"] = gg.make_schedule(lb="edge_only")
    for N in [1 << 18, 1 << 20, 1 << 22]:
        out["pr"]["push-eb-%d" % N] = gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=N)
    for N in [1 << 17, 1 << 18, 1 << 19, 1 << 20, 1 << 21]:
        out["pr"]["pull-strict-eb-%d" % N] = gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True,
                                                              blocking_size=N)
    for lb in ["vp", "etwc", "strict", "twc"]:
        out["bc"]["push-" + lb] = gg.make_schedule(lb=lb)
        s = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
        s.s1.load_balance = gg.LB_NAMES[lb]
        s.threshold = 0.01
        out["bc"]["hybrid-%s-0.01" % lb] = s
    for th in [0.001, 0.01, 0.05]:
        s = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
        s.threshold = th
        out["bc"]["hybrid-etwc-%g" % th] = s
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied %d bytes x3" % (4 * a.numel()))
        return

    import graphgen
    import paper_2012_07990_amd as gg

    torch.cuda.set_device(0)
    t0 = time.time()
    g = graphgen.rmat(args.scale, weights=True)
    src = graphgen.max_degree_vertex(g)
    deg = g.degrees()
    log("graph rmat%d n=%d m=%d built in %.1fs; source %d (degree %d)" %
        (args.scale, g.n, g.m, time.time() - t0, src, deg[src]))
    G = gg.Graph.from_graphgen(g)
    torch.cuda.synchronize()
    scheds = schedules(gg, args.pr_segment)
    # PageRank's EdgeBlocking layout, built once per graph outside the timed step
    # (the paper reports this preprocessing separately)
    pr_eb_ms = G.prepare_pull_blocking(args.pr_segment) if (not args.only or "pr" in args.only.split(",")) else None
    if pr_eb_ms is not None:
        log("PageRank pull EdgeBlocking layout (N = %d) built in %.2f ms" % (args.pr_segment, pr_eb_ms))
    # the EdgeBlocked COO (with weights) that SSSP's dense rounds read, likewise
    sssp_eb_ms = G.prepare_edgeblocking(SSSP_SEGMENT) if (not args.only or "sssp" in args.only.split(",")) else None
    if sssp_eb_ms is not None:
        log("SSSP EdgeBlocked COO (N = %d) built in %.2f ms" % (SSSP_SEGMENT, sssp_eb_ms))
    algos = [a for a in ["bfs", "sssp", "cc", "pr", "bc"] if not args.only or a in args.only.split(",")]
    stream = torch.cuda.current_stream()

    def run(algo, s, stats=None):
        if algo == "bfs":
            return G.bfs(src, s, stats=stats)
        if algo == "sssp":
            return G.sssp(src, s, stats=stats)
        if algo == "cc":
            return G.cc(s, stats=stats)
        if algo == "pr":
            return G.pagerank(s, iters=20, stats=stats)
        return G.bc(src, s, stats=stats)

    if args.counters_sweep:
        marker = torch.ones(1, device="cuda")
        order = []
        for a, d in sweep_schedules(gg).items():
            if a not in algos:
                continue
            for name, s in d.items():
                if args.sweep_filter and not any(f in "%s/%s" % (a, name) for f in args.sweep_filter.split(",")):
                    continue
                try:
                    run(a, s)
                    torch.cuda.synchronize()
                except gg.GGError:
                    continue
                torch.cumsum(marker, 0)
                torch.cuda.synchronize()
                for _ in range(2):
                    run(a, s)
                torch.cuda.synchronize()
                torch.cumsum(marker, 0)
                torch.cuda.synchronize()
                order.append("%s/%s" % (a, name))
        print(json.dumps({"counters_sweep": order, "runs_per_schedule": 2}), flush=True)
        G.close()
        return

    # one run of each algorithm: its outputs are kept on the host and compared
    # with the oracle's (cpu_baseline leg), and they give the traversed-edge
    # numerators
    outs = {}
    for a in algos:
        out = run(a, scheds[a])
        torch.cuda.synchronize()
        outs[a] = tuple(x.cpu().numpy() for x in out) if isinstance(out, tuple) else out.cpu().numpy()
    depth = outs["bfs"] if "bfs" in outs else G.bfs(src, scheds["bfs"]).cpu().numpy()
    reached = depth >= 0
    reached_edges = int(deg[reached].sum())
    edges = {}
    for a in algos:
        edges[a] = {"bfs": reached_edges, "sssp": reached_edges, "bc": reached_edges, "cc": g.m,
                    "pr": 20 * g.m}[a]

    if args.sweep:
        table = {}
        for a, d in sweep_schedules(gg).items():
            if a not in algos:
                continue
            for name, s in d.items():
                if args.sweep_filter and not any(f in "%s/%s" % (a, name) for f in args.sweep_filter.split(",")):
                    continue
                try:
                    run(a, s)
                    torch.cuda.synchronize()
                    ts = []
                    for _ in range(3):
                        st = gg.Stats()
                        t1 = time.perf_counter()
                        run(a, s, st)
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t1)
                    ms = 1e3 * sorted(ts)[1]
                    table["%s/%s" % (a, name)] = ms
                    log("sweep %-28s %9.3f ms  %8.2f GTEPS  iters=%d launches=%d" %
                        (a + "/" + name, ms, edges[a] / ms / 1e6, st.iterations, st.launches))
                except gg.GGError as e:
                    log("sweep %-28s error %s" % (a + "/" + name, e))
        log(json.dumps(table))

    # per-algorithm times (median of 3, after the warm run above)
    per = {}
    for a in algos:
        ts = []
        for _ in range(3):
            st = gg.Stats()
            t1 = time.perf_counter()
            run(a, scheds[a], st)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        ms = 1e3 * sorted(ts)[len(ts) // 2]
        per[a] = {"ms": round(ms, 4), "gteps": round(edges[a] / ms / 1e6, 3), "iterations": st.iterations,
                  "launches": st.launches}
        # work done (outside the timing): edges the traversal examined
        sc = gg.Stats()
        sc.flags = gg.STATS_COUNT_EDGES
        run(a, scheds[a], sc)
        torch.cuda.synchronize()
        per[a]["edges_examined"] = int(sc.edges_examined)
        per[a]["vertices_processed"] = int(sc.vertices_processed)
        b = algorithmic_bytes(a, g, depth, scheds[a], sc)
        per[a]["algorithmic_bytes"] = int(b)
        per[a]["hbm_frac"] = round(b / (ms * 1e-3) / (PEAK_HBM_GBS * 1e9), 4)
        log("algo %-5s %9.3f ms  %8.2f GTEPS  frac %.3f (%s)" % (a, ms, edges[a] / ms / 1e6, per[a]["hbm_frac"],
                                                                  st.as_dict()))

    # the timed steps
    for _ in range(args.warmup):
        for a in algos:
            run(a, scheds[a])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for a in algos:
            run(a, scheds[a])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms_step = 1e3 * wall / args.steps
    step_edges = sum(edges[a] for a in algos)
    value = step_edges / (ms_step * 1e-3) / 1e9

    # roofline of the dominant kernel: the PageRank traversal round
    roof = None
    if "pr" in algos:
        st = gg.Stats()
        st.flags = gg.STATS_TIME_KERNELS
        run("pr", scheds["pr"], st)
        torch.cuda.synchronize()
        per_launch_ms = st.kernel_ms / max(st.kernel_launches, 1)
        # algorithmic bytes of one round: per edge its 4-byte column and the
        # 4-byte contribution it gathers; per (row, source segment) pair with
        # edges, one fp64 accumulator read and written. A launch covers one
        # segment, so a round's bytes are spread over its launches.
        m = g.m
        seg = g.col // args.pr_segment
        chg = np.empty(m, dtype=bool)
        chg[0] = True
        chg[1:] = seg[1:] != seg[:-1]
        chg[g.row_ptr[:-1][deg > 0]] = True
        pairs = int(chg.sum())
        del seg, chg
        launches_per_round = st.kernel_launches / 20.0
        alg_bytes = (8.0 * m + 16.0 * pairs) / launches_per_round
        achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9
        traffic = measured_traffic("paper_2012_07990_amd/csrc/pr.hip", "k_pr_strict_chunks_rmat22.md",
                                   "PULL+STRICT+EB(%d)+LDS(%d)" % (args.pr_segment, PR_LDS_SOURCES))
        # the same rounds with every source gathered from global memory
        st0 = gg.Stats()
        st0.flags = gg.STATS_TIME_KERNELS
        G.pagerank(scheds["pr"], iters=20, stats=st0, lds_cache=False)
        torch.cuda.synchronize()
        plain_ms = st0.kernel_ms / max(st0.kernel_launches, 1)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": st.kernel_name.decode() if isinstance(st.kernel_name, bytes) else str(st.kernel_name),
                "per_launch_ms": round(per_launch_ms, 5), "bytes_per_launch": round(alg_bytes),
                "launches_per_round": launches_per_round, "row_segment_pairs": pairs,
                "lds_cached_sources_per_segment": PR_LDS_SOURCES,
                "per_launch_ms_without_lds_cache": round(plain_ms, 5)}

    tuned = None if args.no_tune else tune_section(gg, G, scheds, run, src, edges, torch, args)

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        cpu, parity = cpu_baseline(g, src, reached_edges, outs, algos)
    G.close()
    del G
    del outs

    small = small_section(gg, graphgen, torch)
    grid = grid_section(gg, graphgen, torch, args.grid, [int(x) for x in args.grid_deltas.split(",")],
                        args.grid_unfused_cap_s) if args.grid else None
    batched = None if args.no_batched else batched_section(gg, graphgen, torch, args)
    serving = None if args.no_serving else serving_section(gg, graphgen, torch, args)
    placement = None if args.no_placement else placement_section(gg, graphgen, torch)

    rec = {
        "metric": "GTEPS per algorithm (BFS/SSSP/CC/PR/BC); batched queries/s + p99 latency",
        "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (BFS/SSSP/CC) + uint64 (BC sigma) + f64 sums of f32 values (PR, BC delta)", "data": "synthetic",
        "config": {"workload": "rmat%d ef16 a.57/b.19/c.19/d.05 symmetrised: BFS(DO)+SSSP(delta)+CC+PR(20)+BC"
                   % args.scale, "n": g.n, "m": g.m, "source": src, "algorithms": algos,
                   "parallelism": "single-gpu"},
        "per_algo": per,
        "preprocessing": {
            **({} if pr_eb_ms is None or "pr" not in per else {
                "pr_pull_edgeblocking_ms": round(pr_eb_ms, 3), "pr_round_ms": round(per["pr"]["ms"] / 20, 4),
                "in_pr_rounds": round(pr_eb_ms / (per["pr"]["ms"] / 20), 2)}),
            **({} if sssp_eb_ms is None else {"sssp_edgeblocked_coo_ms": round(sssp_eb_ms, 1),
                                              "sssp_segment": SSSP_SEGMENT})},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "small": small,
        "tuned": tuned,
        "grid": grid,
        "batched": batched,
        "serving": serving,
        "placement": placement,
    }
    print(json.dumps(rec), flush=True)
    if parity is not None and not parity["all"]:
        log("PARITY FAILURE: the step's GPU outputs differ from the oracle's: %s" % parity)
        sys.exit(1)


def describe(gg, s):
    """Short text form of a schedule."""
    lb = {v: k for k, v in gg.LB_NAMES.items() if k != "vertex_based"}

    def one(x):
        t = "%s %s" % ("pull" if x.direction == gg.PULL else "push", lb.get(x.load_balance, x.load_balance))
        if x.direction == gg.PULL:
            t += " " + ("bitmap" if x.pull_rep == gg.REP_BITMAP else "boolmap")
        if x.delta > 1:
            t += " delta=%d" % x.delta
        if x.edge_blocking:
            t += " EB(%d)" % x.blocking_size
        if x.kernel_fusion:
            t += " fused"
        return t
    return one(s.s1) + (" | hybrid theta=%g -> %s" % (s.threshold, one(s.s2)) if s.hybrid else "")


def small_section(gg, graphgen, torch):
    """R-MAT 14 BFS with the plain vertex-parallel push schedule: a latency-bound
    traversal (the whole graph fits in L2)."""
    g = graphgen.rmat(14)
    G = gg.Graph.from_graphgen(g)
    src = graphgen.max_degree_vertex(g)
    hyb = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    hyb.s1.load_balance = gg.LB_STRICT
    hyb.threshold = 0.01
    rec = {"workload": "rmat14 BFS from the highest-degree vertex %d (degree %d)" % (src, g.degrees()[src]),
           "n": g.n, "m": g.m}
    for key, s in [("push_vp", gg.make_schedule(lb="vp")), ("push_strict", gg.make_schedule(lb="strict")),
                   ("hybrid_strict", hyb)]:
        G.bfs(src, s)
        torch.cuda.synchronize()
        ts = []
        for _ in range(20):
            st = gg.Stats()
            t1 = time.perf_counter()
            d = G.bfs(src, s, stats=st)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        ms = 1e3 * sorted(ts)[len(ts) // 2]
        edges = int(g.degrees()[d.cpu().numpy() >= 0].sum())
        rec[key] = {"schedule": describe(gg, s), "ms": round(ms, 4), "gteps": round(edges / ms / 1e6, 3),
                    "levels": st.iterations, "us_per_level": round(1e3 * ms / max(st.iterations, 1), 2),
                    "launches": st.launches}
    G.close()
    log("small: %s" % rec)
    return rec


def tune_section(gg, G, scheds, run, src, edges, torch, args):
    """The autotuner's pick per algorithm (fixed wall-clock budget) against the
    step's hand-picked schedule, both timed the same way."""
    algo_id = {"bfs": gg.ALGO_BFS, "sssp": gg.ALGO_SSSP, "cc": gg.ALGO_CC, "pr": gg.ALGO_PR, "bc": gg.ALGO_BC}

    def timed(a, s):
        run(a, s)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            run(a, s)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        return 1e3 * sorted(ts)[1]

    out = {"budget_s": args.tune_budget_s, "algos": {}}
    for a in ["bfs", "sssp", "cc", "pr", "bc"]:
        t0 = time.perf_counter()
        s, best = G.autotune(algo_id[a], args.tune_budget_s, [src])
        took = time.perf_counter() - t0
        ms_t, ms_h = timed(a, s), timed(a, scheds[a])
        rec = {"tuned": describe(gg, s), "tuned_ms": round(ms_t, 3), "bench_schedule": describe(gg, scheds[a]),
               "bench_ms": round(ms_h, 3), "tuner_s": round(took, 1)}
        log("tune %s: %s" % (a, rec))
        out["algos"][a] = rec
    return out


def grid_section(gg, graphgen, torch, W, deltas, unfused_cap_s):
    """High-diameter road-like grid (the kernel-fusion experiment's setting):
    BFS and delta-stepping SSSP over the given deltas from the corner vertex,
    each as one persistent launch (fused) and as one launch per round
    (unfused; skipped when the fused run already took longer than
    unfused_cap_s, since the unfused loop is several times slower). Every
    delta and both forms must give the same distances (and BFS depths)."""
    import numpy as np
    g = graphgen.grid(W)
    G = gg.Graph.from_graphgen(g)
    out = {"workload": "grid %dx%d, 10%% non-tree edges dropped, weights 1..999, source 0" % (W, W),
           "n": g.n, "m": g.m, "unfused_cap_s": unfused_cap_s, "runs": []}
    # first calls allocate the workspaces (outside every timing)
    G.bfs(0, gg.make_schedule(lb="cm", fusion=True))
    G.sssp(0, gg.make_schedule(lb="cm", delta=4096, fusion=True))
    G.sssp(0, gg.make_schedule(lb="cm", delta=4096))
    torch.cuda.synchronize()
    first = {}
    identical = True
    for algo in ["bfs", "sssp"]:
        for delta in (deltas if algo == "sssp" else [0]):
            fused_ms = 0.0
            for fused in (True, False):
                if not fused and fused_ms > 1e3 * unfused_cap_s:
                    log("grid: %s delta %d unfused skipped (fused run took %.1f s)" % (algo, delta, fused_ms / 1e3))
                    continue
                sch = gg.make_schedule(lb="cm", delta=max(delta, 1), fusion=fused)

                def run(st):
                    return G.sssp(0, sch, stats=st) if algo == "sssp" else G.bfs(0, sch, stats=st)
                ts = []
                for rep in range(3):
                    st = gg.Stats()
                    t1 = time.perf_counter()
                    d = run(st)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t1)
                    if ts[-1] > 2.0:  # long runs are timed once
                        break
                ms = 1e3 * sorted(ts)[len(ts) // 2]
                d = d.cpu().numpy()
                if algo not in first:
                    first[algo] = d
                same = bool(np.array_equal(d, first[algo]))
                identical &= same
                rec = {"algo": algo, "delta": delta if algo == "sssp" else None, "fused": fused, "ms": round(ms, 3),
                       "rounds": st.iterations, "buckets": st.buckets, "launches": st.launches,
                       "us_per_round": round(1e3 * ms / max(st.iterations, 1), 2),
                       "us_per_bucket": round(1e3 * ms / st.buckets, 2) if st.buckets else None,
                       "timed_runs": len(ts), "same_as_first": same}
                log("grid: %s" % rec)
                out["runs"].append(rec)
                if fused:
                    fused_ms = ms
    out["identical_across_deltas_and_forms"] = identical
    G.close()
    return out


def batched_section(gg, graphgen, torch, args):
    """64 BFS + 16 BC sources on R-MAT 20 in one batched call each, against the
    same sources as single-source calls (bit-identity checked on the way). The
    autotuner picks the BFS and BC schedules on this graph (load balance,
    direction and threshold); the single calls run them, and the batched
    calls take their form from the picked direction."""
    import numpy as np
    g = graphgen.rmat(20, weights=True)
    G = gg.Graph.from_graphgen(g)
    deg = g.degrees()
    bfs_src = graphgen.sample_giant_sources(g, 64, 7)
    bc_src = bfs_src[:16]
    tuner = None
    if args.no_tune:
        sb = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
        sb.threshold = 0.01
        sc = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
        sc.threshold = 0.01
    else:
        t0 = time.perf_counter()
        sb, _ = G.autotune(gg.ALGO_BFS, args.tune_budget_s, [int(x) for x in bfs_src[:8]])
        sc, _ = G.autotune(gg.ALGO_BC, args.tune_budget_s, [int(x) for x in bc_src[:8]])
        tuner = {"bfs": describe(gg, sb), "bc": describe(gg, sc), "tuner_s": round(time.perf_counter() - t0, 1)}
        log("batched: tuned schedules %s" % tuner)

    def timed(f, reps=3):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        return sorted(ts)[len(ts) // 2]

    # one persistent launch per batch: 64 BFS sources, then the 16 BC sources,
    # in the tuned schedules' forms with kernel fusion
    def fused(s):
        f = gg.make_schedule()
        f.hybrid, f.threshold, f.s1, f.s2 = s.hybrid, s.threshold, s.s1, s.s2
        f.s1.kernel_fusion = 1
        return f
    mb = fused(sb)
    mc = fused(sc)
    d_multi = G.bfs_multi(bfs_src, mb)
    s_multi, dl_multi = G.bc_multi(bc_src, mc)
    ok = True
    for i in range(0, 64, 9):
        ok &= bool(torch.equal(d_multi[i], G.bfs(int(bfs_src[i]), sb)))
    for i in range(0, 16, 5):
        s1, d1 = G.bc(int(bc_src[i]), sc)
        ok &= bool(torch.equal(s_multi[i], s1)) and bool(torch.equal(dl_multi[i].view(torch.int32),
                                                                        d1.view(torch.int32)))
    t_multi = timed(lambda: (G.bfs_multi(bfs_src, mb), G.bc_multi(bc_src, mc)))
    # the same batches with one launch per level (host-driven loop)
    mb_l, mc_l = sb, sc
    t_levels = timed(lambda: (G.bfs_multi(bfs_src, mb_l), G.bc_multi(bc_src, mc_l)))
    # the single-call baseline runs the faster of the tuned and the preset
    # schedule per algorithm (timed on 8 of the sources)
    def faster(run, cands, srcs):
        best = None
        for s in cands:
            run(int(srcs[0]), s)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for x in srcs[:8]:
                run(int(x), s)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            if best is None or dt < best[0]:
                best = (dt, s)
        return best[1]
    pb = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    pb.threshold = 0.01
    pc = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
    pc.threshold = 0.01
    sb1 = faster(lambda x, s: G.bfs(x, s), [sb, pb], bfs_src)
    sc1 = faster(lambda x, s: G.bc(x, s), [sc, pc], bc_src)
    t_single = timed(lambda: ([G.bfs(int(x), sb1) for x in bfs_src], [G.bc(int(x), sc1) for x in bc_src]), reps=1)
    reach = d_multi.cpu().numpy() >= 0
    edges = float(sum(deg[reach[i]].sum() for i in range(64)))
    reach_bc = s_multi.cpu().numpy() != 0
    edges += float(sum(deg[reach_bc[i]].sum() for i in range(16)))
    t_best = min(t_multi, t_levels)
    log("batched: persistent %.2f ms, launch per level %.2f ms, single %.2f ms, speedup %.2fx, identical=%s" %
        (t_multi * 1e3, t_levels * 1e3, t_single * 1e3, t_single / t_best, ok))
    out = {"workload": "rmat20: 64 BFS + 16 BC sources (uniform over the largest component, seed 7)",
           "ms_batched": round(t_best * 1e3, 3), "ms_batched_persistent": round(t_multi * 1e3, 3),
           "ms_batched_launch_per_level": round(t_levels * 1e3, 3), "ms_single_calls": round(t_single * 1e3, 3),
           "speedup": round(t_single / t_best, 2), "gteps_batched": round(edges / t_best / 1e9, 2),
           "queries_per_s": round(80 / t_best, 1), "bit_identical": ok,
           "schedules": {"bfs": describe(gg, sb), "bc": describe(gg, sc)},
           "single_call_schedules": {"bfs": describe(gg, sb1), "bc": describe(gg, sc1)}, "tuner": tuner}
    # 64 SSSP sources: on R-MAT 20 and on the 2048^2 grid, each form with its
    # fastest delta (batched 64 / single STRICT 4096 on R-MAT; 4096 for both on
    # the grid), against single calls (on the grid 4 single calls stand for the 64)
    out["sssp"] = []
    for name, Gx, srcs, single_s, ms_delta, nsingle in [
            ("rmat20", G, bfs_src, gg.make_schedule(lb="strict", delta=4096), 64, 64),
            ("grid2048", None, None, gg.make_schedule(lb="cm", delta=4096, fusion=True), 4096, 4)]:
        if Gx is None:
            gh = graphgen.grid(2048)
            Gx = gg.Graph.from_graphgen(gh)
            srcs = graphgen.sample_giant_sources(gh, 64, 7)
        ms_s = gg.make_schedule(delta=ms_delta)
        st = gg.Stats()
        dm = Gx.sssp_multi(srcs, ms_s, stats=st)
        ok_s = all(bool(torch.equal(dm[i], Gx.sssp(int(srcs[i]), single_s))) for i in range(0, 64, 21))
        t_m = timed(lambda: Gx.sssp_multi(srcs, ms_s), reps=1 if name.startswith("grid") else 3)
        t_1 = timed(lambda: [Gx.sssp(int(x), single_s) for x in srcs[:nsingle]], reps=1) * 64 / nsingle
        rec = {"graph": name, "k": 64, "delta_batched": ms_delta, "delta_single": int(single_s.s1.delta),
               "ms_batched": round(t_m * 1e3, 3),
               "ms_single_calls": round(t_1 * 1e3, 3), "single_calls_timed": nsingle,
               "speedup": round(t_1 / t_m, 2), "rounds": st.iterations, "buckets": st.buckets,
               "queries_per_s": round(64 / t_m, 1), "bit_identical": ok_s}
        log("batched sssp: %s" % rec)
        out["sssp"].append(rec)
        if name.startswith("grid"):
            # 64 BFS sources on the grid: the push loop against the pull sweep
            # and against single fused BFS calls (4 timed, scaled to 64)
            bs = gg.make_schedule(lb="cm", fusion=True)
            pull = gg.make_schedule(direction=gg.PULL)
            st = gg.Stats()
            dp = Gx.bfs_multi(srcs, gg.make_schedule(), stats=st)
            ok_b = bool(torch.equal(dp, Gx.bfs_multi(srcs, pull)))
            ok_b &= all(bool(torch.equal(dp[i], Gx.bfs(int(srcs[i]), bs))) for i in range(0, 64, 21))
            t_push = timed(lambda: Gx.bfs_multi(srcs, gg.make_schedule()), reps=1)
            t_pull = timed(lambda: Gx.bfs_multi(srcs, pull), reps=1)
            t_1 = timed(lambda: [Gx.bfs(int(x), bs) for x in srcs[:4]], reps=1) * 16
            rec = {"graph": name, "k": 64, "ms_push_batched": round(t_push * 1e3, 3),
                   "ms_pull_batched": round(t_pull * 1e3, 3), "ms_single_calls": round(t_1 * 1e3, 3),
                   "single_calls_timed": 4, "speedup": round(t_1 / min(t_push, t_pull), 2), "levels": st.iterations,
                   "queries_per_s": round(64 / min(t_push, t_pull), 1), "bit_identical": ok_b}
            log("batched bfs: %s" % rec)
            out["grid_bfs"] = rec
        Gx.close()
    return out


def serving_section(gg, graphgen, torch, args):
    """Poisson streams of mixed BFS/SSSP/BC queries over four resident graphs
    (R-MAT 18, 20 and 23 with weights, and the 2048^2 road-like grid), served
    with continuous batching, against one query per launch in arrival order
    on the same GPU under the same per-(graph, algorithm) schedules."""
    import numpy as np
    specs = [("rmat18", lambda: graphgen.rmat(18, weights=True)),
             ("rmat20", lambda: graphgen.rmat(20, weights=True)),
             ("rmat23", lambda: graphgen.rmat(23, weights=True)),
             ("grid2048", lambda: graphgen.grid(2048))]
    Gs, cand, names = [], [], []
    for name, f in specs:
        t0 = time.perf_counter()
        g = f()
        Gs.append(gg.Graph.from_graphgen(g))
        cand.append(graphgen.giant_component(g))
        names.append(name)
        log("serving: %s n=%d m=%d ready in %.1fs" % (name, g.n, g.m, time.perf_counter() - t0))
        del g
    is_rmat = [nm.startswith("rmat") for nm in names]
    step = schedules(gg)
    sched = []
    for gi in range(len(Gs)):
        if is_rmat[gi]:
            sched.append({gg.ALGO_BFS: step["bfs"], gg.ALGO_SSSP: step["sssp"], gg.ALGO_BC: step["bc"]})
        else:  # high diameter: persistent loops, wide buckets
            sched.append({gg.ALGO_BFS: gg.make_schedule(lb="cm", fusion=True),
                          gg.ALGO_SSSP: gg.make_schedule(lb="cm", delta=4096, fusion=True)})
    rates = [float(x) for x in args.serve_rates.split(",")]
    rng = np.random.default_rng(11)
    algo_name = {gg.ALGO_BFS: "bfs", gg.ALGO_SSSP: "sssp", gg.ALGO_BC: "bc"}

    def make_stream(rate, seconds):
        k = max(1, int(rate * seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=k))
        qs = []
        for t in arrivals:
            gi = int(rng.integers(0, len(Gs)))
            u = rng.random()
            algo = gg.ALGO_BFS if u < 0.5 else (gg.ALGO_SSSP if u < 0.85 else gg.ALGO_BC)
            if algo == gg.ALGO_BC and not is_rmat[gi]:
                algo = gg.ALGO_BFS
            src = int(cand[gi][int(rng.integers(0, cand[gi].size))])
            qs.append((float(t), gi, algo, src))
        return qs

    def pct(xs, p):
        return round(float(np.percentile(np.asarray(xs), p)), 3) if len(xs) else None

    def serve(qs, budget):
        srv = gg.Server(budget_bytes=budget, nstreams=4)
        gids = [srv.add_graph(G) for G in Gs]
        for gi in range(len(Gs)):
            for a, sc in sched[gi].items():
                srv.set_schedule(gids[gi], a, sc)
        t0 = time.perf_counter()
        tickets = []
        for (ta, gi, algo, src) in qs:
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            tickets.append((srv.submit(gids[gi], algo, src), algo))
        lat = {a: [] for a in algo_name}
        done = 0
        for i, (t, algo) in enumerate(tickets):
            r = srv.wait(t, 60.0)
            if r is None:
                log("serving: query %d still running after 60 s, stopping the wait" % i)
                break
            lat[algo].append(r["latency_ms"])
            done += 1
        t_end = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return done, t_end, lat, st

    def baseline(qs, cap_s):
        t1 = time.perf_counter()
        lat = []
        for (ta, gi, algo, src) in qs:
            now = time.perf_counter() - t1
            if now > cap_s:
                break
            if ta > now:
                time.sleep(ta - now)
            G, sc = Gs[gi], sched[gi][algo]
            if algo == gg.ALGO_BFS:
                G.bfs(src, sc)
            elif algo == gg.ALGO_SSSP:
                G.sssp(src, sc)
            else:
                G.bc(src, sc)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1 - ta) * 1e3)
        return len(lat), time.perf_counter() - t1, lat

    budget = 16 << 30
    out = {"graphs": names, "mix": "BFS 50% / SSSP 35% / BC 15% (BC on R-MAT only); graph uniform; source uniform "
                                   "over the graph's largest component",
           "budget_bytes": budget, "streams": 4, "seconds_per_rate": args.serve_seconds,
           "schedules": {nm: {algo_name[a]: describe(gg, sc) for a, sc in sched[gi].items()}
                         for gi, nm in enumerate(names)}, "rates": []}
    # warm-up: every (graph, algorithm) once through the server and once alone
    warm = [(0.0, gi, a, int(cand[gi][0])) for gi in range(len(Gs)) for a in sched[gi]]
    serve(warm, budget)
    baseline(warm, 1e9)
    sec0 = time.perf_counter()
    for rate in rates:
        if time.perf_counter() - sec0 > args.serve_budget_s:
            log("serving: wall-clock cap reached, rate %g skipped" % rate)
            break
        qs = make_stream(rate, args.serve_seconds)
        log("serving: rate %g, %d queries" % (rate, len(qs)))
        done, t_end, lat, st = serve(qs, budget)
        served_qps = done / t_end
        nb, tb, blat = baseline(qs, args.serve_baseline_s)
        base_qps = nb / tb
        alll = sum(lat.values(), [])
        rec = {"rate_qps": rate, "queries": len(qs), "completed": done, "served_qps": round(served_qps, 1),
               "sustained": served_qps >= 0.95 * min(rate, len(qs) / max(qs[-1][0], 1e-9)),
               "p50_ms": pct(alll, 50), "p99_ms": pct(alll, 99),
               "per_algo": {algo_name[a]: {"queries": len(v), "p50_ms": pct(v, 50), "p99_ms": pct(v, 99)}
                            for a, v in lat.items() if v},
               "max_batch": st["max_batch"], "batches": st["batches"], "bytes_peak": st["bytes_peak"],
               "baseline_qps": round(base_qps, 1), "baseline_p50_ms": pct(blat, 50),
               "baseline_p99_ms": pct(blat, 99), "baseline_queries": nb,
               "throughput_ratio": round(served_qps / base_qps, 2)}
        log("serving rate %g: %s" % (rate, rec))
        out["rates"].append(rec)
    for G in Gs:
        G.close()
    return out


def placement_section(gg, graphgen, torch):
    """The CPU backend (the library's threads on the host CSR) against the GPU
    on the same query, and the placement gg_place picks: delta-stepping SSSP
    and BFS on the 2048^2 road-like grid and on R-MAT 20 (the paper's CPU-vs-GPU
    comparison is delta-stepping on road graphs)."""
    import numpy as np
    _, nproc = host_cpu()
    out = {"threads": nproc, "runs": []}
    for name, make in [("grid2048", lambda: graphgen.grid(2048)), ("rmat20", lambda: graphgen.rmat(20, weights=True))]:
        g = make()
        G = gg.Graph.from_graphgen(g)
        C = gg.CpuGraph.from_graphgen(g)
        src = 0 if name.startswith("grid") else graphgen.max_degree_vertex(g)
        grid = name.startswith("grid")
        for algo, s in [(gg.ALGO_SSSP, gg.make_schedule(lb="cm", delta=4096, fusion=True) if grid
                         else gg.make_schedule(lb="strict", delta=4096)),
                        (gg.ALGO_BFS, gg.make_schedule(lb="cm", fusion=True) if grid else schedules(gg)["bfs"])]:
            target, gpu_ms, cpu_ms = gg.place(G, C, algo, s, src, nthreads=nproc)
            same = bool(np.array_equal(G.sssp(src, s).cpu().numpy(), C.sssp(src, 4096)) if algo == gg.ALGO_SSSP
                        else np.array_equal(G.bfs(src, s).cpu().numpy(), C.bfs(src)))
            rec = {"graph": name, "algo": "sssp" if algo == gg.ALGO_SSSP else "bfs", "gpu_schedule": describe(gg, s),
                   "gpu_ms": round(gpu_ms, 3), "cpu_ms": round(cpu_ms, 3),
                   "target": "cpu" if target == gg.TARGET_CPU else "gpu", "identical": same}
            log("placement: %s" % rec)
            out["runs"].append(rec)
        C.close()
        G.close()
    return out


def host_cpu():
    """(CPU model, logical CPUs this process may run on)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return model, avail


def gg_lb_edge_only():
    import paper_2012_07990_amd as gg
    return gg.LB_EDGE_ONLY


def algorithmic_bytes(algo, g, depth, sched, st):
    """Bytes the method itself must move for one run (the per-vertex and
    per-edge figures of the byte model in the design doc), from the run's device
    counters (examined edges, processed vertices) and the BFS level structure.
    Hybrid runs: a level whose input frontier holds more than threshold * n
    vertices is a PULL level (the HybridGPUSchedule rule); its edges are the
    examined edges the PUSH levels do not account for."""
    import numpy as np
    n, m = g.n, g.m
    deg = g.degrees()
    E, V = float(st.edges_examined), float(st.vertices_processed)
    if algo == "sssp":
        return 20.0 * V + 12.0 * E
    if algo == "cc":
        if sched.s1.load_balance == gg_lb_edge_only():
            # EDGE_ONLY sweeps every undirected edge once as a (u, v) pair:
            # 8 bytes of pair plus the two labels per pair, and per vertex the
            # shortcut's label read and write
            return 8.0 * V + 16.0 * E
        return 12.0 * V + 8.0 * E
    if algo == "pr":
        return 20.0 * (16.0 * n + 8.0 * m)
    # BFS and BC forward: replay the direction choice level by level
    reached = depth >= 0
    levels = int(depth.max()) + 1
    F = np.bincount(depth[reached], minlength=levels).astype(np.float64)
    Fe = np.bincount(depth[reached], weights=deg[reached].astype(np.float64), minlength=levels)
    visited = np.cumsum(F)
    push_b, pull_b, e_push = 0.0, 0.0, 0.0
    for L in range(levels):
        pull = bool(sched.hybrid) and F[L] > float(sched.threshold) * n
        if pull:
            pull_b += 12.0 * (n - visited[L]) + n / 8.0
        else:
            push_b += 20.0 * F[L]
            e_push += Fe[L]
    e_pull = max(E - e_push, 0.0)
    fwd = push_b + 8.0 * e_push + pull_b + 4.125 * e_pull
    if algo == "bfs":
        return fwd
    # BC: sigma per vertex and per examined edge forward; backward over every
    # reached vertex's edges (column, depth, sigma, delta) and its delta
    e_back = float(deg[reached].sum())
    return fwd + 8.0 * float(reached.sum()) + 8.0 * E + 20.0 * e_back + 4.0 * float(reached.sum())


def cpu_baseline(g, src, reached_edges, outs, algos):
    """The oracle (single-threaded C, one core) on the step's whole workload:
    the same graph and source, PageRank for all 20 rounds. Its outputs are the
    reference the step's GPU outputs are compared with (depths, distances,
    labels and path counts bit for bit; PageRank within max-abs 1e-6 and the
    sum, L1 and relative checks; BC dependencies within relative 1e-4)."""
    import numpy as np
    import oracle
    model, avail = host_cpu()
    csr_code = oracle.check_csr(g.n, g.row_ptr, g.col)  # re-validation, not timed
    calls = {"bfs": lambda: oracle.bfs(g.n, g.row_ptr, g.col, src),
             "sssp": lambda: oracle.sssp(g.n, g.row_ptr, g.col, g.w, src),
             "cc": lambda: oracle.cc(g.n, g.row_ptr, g.col),
             "pr": lambda: oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20),
             "bc": lambda: oracle.bc(g.n, g.row_ptr, g.col, src)}
    t, ref = {}, {}
    for a in algos:
        t0 = time.perf_counter()
        ref[a] = calls[a]()
        t[a] = time.perf_counter() - t0
    step_s = sum(t.values())
    step_edges = sum({"bfs": reached_edges, "sssp": reached_edges, "bc": reached_edges, "cc": g.m,
                      "pr": 20 * g.m}[a] for a in algos)
    par = {"csr_check": csr_code == 0}
    for a in algos:
        got, exp = outs[a], ref[a]
        if a in ("bfs", "sssp", "cc"):
            par[a] = bool(np.array_equal(got, exp))
        elif a == "pr":
            err = np.abs(got.astype(np.float64) - exp)
            par[a] = bool(err.max() <= 1e-6 and err.sum() <= 1e-4 and (err / exp).max() <= 1e-3
                          and abs(float(got.astype(np.float64).sum()) - 1.0) <= 1e-4)
            par["pr_max_abs"] = float(err.max())
        else:
            sig, dl = got
            es, ed = exp
            ok_s = bool(np.array_equal(sig.view(np.uint64), es))
            rel = np.abs(dl.astype(np.float64) - ed)
            ok_d = bool((rel <= 1e-4 * np.abs(ed) + 1e-6).all())
            par[a] = ok_s and ok_d
    par["all"] = all(v for k, v in par.items() if isinstance(v, bool))
    log("parity against the oracle: %s" % par)
    cpu = {"value": round(step_edges / step_s / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
           "nproc": avail, "cpu_model": model,
           "sample": "one full step (%s) on the same graph and source, PageRank for all 20 rounds, one core (%s)" %
                     ("+".join(algos), ", ".join("%s %.2fs" % (a, t[a]) for a in algos))}
    return cpu, par


if __name__ == "__main__":
    import atexit
    # registered before the library is imported, so it runs after the
    # library's own exit hook has closed every graph and server
    atexit.register(_report_exit)
    main()
