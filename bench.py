"""Benchmark: GTEPS of the five traversal algorithms on a synthetic R-MAT
scale-22 graph (4,194,304 vertices, edge factor 16, a/b/c/d = .57/.19/.19/.05,
symmetrised, self-loops and duplicates removed) on one MI355X.

One step = one pass of the whole hot path over the resident graph:
direction-optimising BFS, delta-stepping SSSP, CC (hooking + shortcutting),
PageRank (FP32, 20 rounds, d = 0.85) and single-source BC, each under its
tuned schedule. `value` is the aggregate GTEPS of the step: traversed edges
(BFS/SSSP/BC: sum of degrees of reached vertices; CC: m; PR: 20 m) over the
step's wall time with the graph already in HBM.

Prints ONE JSON line (rank 0). `--gpus N` with N > 1 is refused: this build
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

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--only", default="", help="comma list of algorithms to run (bfs,sssp,cc,pr,bc)")
    p.add_argument("--sweep", action="store_true", help="time every schedule family per algorithm")
    p.add_argument("--verbose", action="store_true")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def schedules(gg):
    """The schedule each algorithm runs in the step (chosen by sweeps on this graph family)."""
    bfs = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    bfs.threshold = 0.01
    sssp = gg.make_schedule(lb="etwc", delta=64)
    cc = gg.make_schedule(lb="etwc")
    pr = gg.make_schedule(lb="strict", direction=gg.PULL)
    bc = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
    bc.threshold = 0.01
    return {"bfs": bfs, "sssp": sssp, "cc": cc, "pr": pr, "bc": bc}


def sweep_schedules(gg):
    out = {"bfs": {}, "sssp": {}, "cc": {}, "pr": {}, "bc": {}}
    for lb in ["vp", "wm", "cm", "strict", "twc", "etwc"]:
        out["bfs"]["push-" + lb] = gg.make_schedule(lb=lb)
        out["cc"][lb] = gg.make_schedule(lb=lb)
    out["cc"]["edge_only"] = gg.make_schedule(lb="edge_only")
    for th in [0.001, 0.01, 0.05, 0.2]:
        s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_BFS_HYBRID)
        s.threshold = th
        out["bfs"]["hybrid-vp-%g" % th] = s
        s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
        s.threshold = th
        out["bfs"]["hybrid-etwc-%g" % th] = s
    out["bfs"]["fused-vp"] = gg.make_schedule(lb="vp", fusion=True)
    out["bfs"]["fused-hybrid"] = gg.make_schedule(lb="vp", fusion=True, threshold=0.01,
                                                  hybrid={"direction": gg.PULL, "pull_rep": gg.REP_BITMAP})
    for d in [1, 8, 64, 512, 4096]:
        for lb in ["vp", "etwc", "cm"]:
            out["sssp"]["%s-d%d" % (lb, d)] = gg.make_schedule(lb=lb, delta=d)
        out["sssp"]["fused-etwc-d%d" % d] = gg.make_schedule(lb="etwc", delta=d, fusion=True)
    for lb in ["vp", "wm", "etwc", "strict"]:
        out["pr"]["pull-" + lb] = gg.make_schedule(lb=lb, direction=gg.PULL)
    out["pr"]["push-edge"] = gg.make_schedule(lb="edge_only")
    for N in [1 << 18, 1 << 20, 1 << 22]:
        out["pr"]["push-eb-%d" % N] = gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=N)
    for N in [1 << 17, 1 << 18, 1 << 19, 1 << 20, 1 << 21]:
        out["pr"]["pull-strict-eb-%d" % N] = gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True,
                                                              blocking_size=N)
    for lb in ["vp", "etwc"]:
        out["bc"]["push-" + lb] = gg.make_schedule(lb=lb)
    for th in [0.001, 0.01, 0.05]:
        s = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
        s.threshold = th
        out["bc"]["hybrid-etwc-%g" % th] = s
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

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
    scheds = schedules(gg)
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

    # traversed-edge numerators from one verified run of each algorithm
    reached = None
    edges = {}
    for a in algos:
        out = run(a, scheds[a])
        torch.cuda.synchronize()
        if a == "bfs":
            reached = out.cpu().numpy() >= 0
    if reached is None:
        d = G.bfs(src, scheds["bfs"]).cpu().numpy()
        reached = d >= 0
    reached_edges = int(deg[reached].sum())
    for a in algos:
        edges[a] = {"bfs": reached_edges, "sssp": reached_edges, "bc": reached_edges, "cc": g.m,
                    "pr": 20 * g.m}[a]

    if args.sweep:
        table = {}
        for a, d in sweep_schedules(gg).items():
            if a not in algos:
                continue
            for name, s in d.items():
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
        log("algo %-5s %9.3f ms  %8.2f GTEPS  (%s)" % (a, ms, edges[a] / ms / 1e6, st.as_dict()))

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
        n, m = g.n, g.m
        alg_bytes = 8.0 * m + 16.0 * n  # per round: col + contrib gather per edge; row_ptr, rank, contrib per vertex
        achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": st.kernel_name.decode() if isinstance(st.kernel_name, bytes) else str(st.kernel_name),
                "per_launch_ms": round(per_launch_ms, 5), "bytes_per_launch": alg_bytes}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, src, reached_edges)

    rec = {
        "metric": "GTEPS per algorithm (BFS/SSSP/CC/PR/BC); batched queries/s + p99 latency",
        "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (BFS/SSSP/CC/BC sigma) + f32 (PR, BC delta)", "data": "synthetic",
        "config": {"workload": "rmat%d ef16 a.57/b.19/c.19/d.05 symmetrised: BFS(DO)+SSSP(delta)+CC+PR(20)+BC"
                   % args.scale, "n": g.n, "m": g.m, "source": src, "algorithms": algos,
                   "parallelism": "single-gpu"},
        "per_algo": per,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    G.close()


def cpu_baseline(g, src, reached_edges):
    """The oracle (single-threaded C) on a bounded sample of the same workload."""
    import oracle
    t = {}
    t0 = time.perf_counter(); oracle.bfs(g.n, g.row_ptr, g.col, src); t["bfs"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.cc(g.n, g.row_ptr, g.col); t["cc"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 2); t["pr2"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.sssp(g.n, g.row_ptr, g.col, g.w, src); t["sssp"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.bc(g.n, g.row_ptr, g.col, src); t["bc"] = time.perf_counter() - t0
    step_s = t["bfs"] + t["cc"] + 10 * t["pr2"] + t["sssp"] + t["bc"]
    step_edges = 3 * reached_edges + g.m + 20 * g.m
    return {"value": round(step_edges / step_s / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "one full step on the same graph and source, PageRank timed for 2 rounds and scaled to 20 "
                      "(bfs %.2fs, cc %.2fs, pr2 %.2fs, sssp %.2fs, bc %.2fs)" %
                      (t["bfs"], t["cc"], t["pr2"], t["sssp"], t["bc"])}


if __name__ == "__main__":
    main()
