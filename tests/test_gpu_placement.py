"""CPU-or-GPU placement through the C ABI (the query timed on both backends,
the faster kept on the graph), and the two backends' outputs side by side:
depths, distances, labels and path counts identical, PageRank and BC
dependencies within the GPU tolerances of each other."""
import ctypes

import numpy as np
import pytest

import graphgen
import paper_2012_07990_amd as gg
from gpu_util import dev_graph, host_graph, source

pytestmark = pytest.mark.gpu

CASES = [("rmat12", gg.ALGO_BFS, lambda: gg.make_schedule(lb="strict")),
         ("rmat12", gg.ALGO_SSSP, lambda: gg.make_schedule(lb="strict", delta=4096)),
         ("grid64", gg.ALGO_SSSP, lambda: gg.make_schedule(lb="cm", delta=512, fusion=True)),
         ("grid64", gg.ALGO_BFS, lambda: gg.make_schedule(lb="cm", fusion=True)),
         ("rmat12", gg.ALGO_CC, lambda: gg.make_schedule(lb="edge_only")),
         ("rmat12", gg.ALGO_PR, lambda: gg.make_schedule(lb="strict", direction=gg.PULL)),
         ("star5000", gg.ALGO_BC, lambda: gg.make_schedule(lb="etwc"))]


@pytest.mark.parametrize("name,algo,sched", CASES)
def test_place_and_backends_agree(name, algo, sched):
    g = host_graph(name)
    G = dev_graph(name)
    C = gg.CpuGraph.from_graphgen(g)
    s = sched()
    src = source(name)
    target, gpu_ms, cpu_ms = gg.place(G, C, algo, s, src, nthreads=8)
    assert target in (gg.TARGET_GPU, gg.TARGET_CPU) and gpu_ms > 0 and cpu_ms > 0
    assert target == (gg.TARGET_CPU if cpu_ms < gpu_ms else gg.TARGET_GPU)
    t = ctypes.c_int32()
    assert gg._lib.gg_placement_get(G.handle, algo, ctypes.byref(t)) == gg.OK and t.value == target
    if algo == gg.ALGO_BFS:
        assert np.array_equal(G.bfs(src, s).cpu().numpy(), C.bfs(src))
    elif algo == gg.ALGO_SSSP:
        assert np.array_equal(G.sssp(src, s).cpu().numpy(), C.sssp(src, s.s1.delta))
    elif algo == gg.ALGO_CC:
        assert np.array_equal(G.cc(s).cpu().numpy(), C.cc())
    elif algo == gg.ALGO_PR:
        a, b = G.pagerank(s).cpu().numpy().astype(np.float64), C.pagerank().astype(np.float64)
        assert np.abs(a - b).max() <= 2e-6
    else:
        sg, dg = G.bc(src, s)
        sc, dc = C.bc(src)
        assert np.array_equal(sg.cpu().numpy().view(np.uint64), sc)
        dg = dg.cpu().numpy().astype(np.float64)
        assert (np.abs(dg - dc) <= 2e-4 * np.abs(dc) + 2e-6).all()


def test_placement_unknown_before_place():
    G = gg.Graph.from_graphgen(graphgen.path(10))
    t = ctypes.c_int32()
    assert gg._lib.gg_placement_get(G.handle, gg.ALGO_BFS, ctypes.byref(t)) == gg.ERR_NOT_FOUND
    G.close()
