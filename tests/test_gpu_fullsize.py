"""GPU parity at the benchmark's full sizes, in the schedules the benchmark times.

* R-MAT scale 22 (4,194,304 vertices, ~128M directed entries): the benchmark
  step's direction-optimising BFS, delta-stepping SSSP, CC, 20 PageRank
  rounds and single-source BC from the highest-degree vertex.
* R-MAT scale 20: 64 batched BFS sources and 16 batched BC sources, as one
  persistent launch per batch and as one launch per level.
* 4096 x 4096 road-like grid: fused and unfused BFS and delta-stepping SSSP
  from the corner vertex.

Every output is compared element by element with the CPU oracle: depths,
distances, labels and path counts bit for bit; PageRank within max-abs 1e-6
plus the sum, L1 and relative checks; BC dependencies within relative 1e-4.
Every input is re-validated by the oracle's CSR check first.
"""
import functools

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import HAS_GPU, assert_int_equal

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAS_GPU, reason="needs a GPU")]

if HAS_GPU:
    import torch
    import paper_2012_07990_amd as gg
    import bench


@functools.lru_cache(maxsize=None)
def big(name):
    if name == "rmat22":
        g = graphgen.rmat(22, weights=True)
    elif name == "rmat20":
        g = graphgen.rmat(20, weights=True)
    elif name == "grid4096":
        g = graphgen.grid(4096)
    else:
        raise KeyError(name)
    print("built %s n=%d m=%d" % (name, g.n, g.m), flush=True)
    assert oracle.check_csr(g.n, g.row_ptr, g.col) == 0
    return g


@functools.lru_cache(maxsize=None)
def dev(name):
    g = big(name)
    return gg.Graph.from_graphgen(g)


@functools.lru_cache(maxsize=None)
def ref(name, algo, src=None):
    g = big(name)
    if algo == "bfs":
        return oracle.bfs(g.n, g.row_ptr, g.col, src)
    if algo == "sssp":
        return oracle.sssp(g.n, g.row_ptr, g.col, g.w, src)
    if algo == "cc":
        return oracle.cc(g.n, g.row_ptr, g.col)
    if algo == "pr":
        return oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20)
    if algo == "bc":
        return oracle.bc(g.n, g.row_ptr, g.col, src)
    raise KeyError(algo)


def step_schedules():
    return bench.schedules(gg)


def check_pr(got, exp):
    err = np.abs(got.astype(np.float64) - exp)
    assert err.max() <= 1e-6, err.max()
    assert err.sum() <= 1e-4, err.sum()
    assert (err / exp).max() <= 1e-3
    assert abs(float(got.astype(np.float64).sum()) - 1.0) <= 1e-4


def check_bc(sig, dl, exp_sig, exp_dl, what):
    assert_int_equal(sig.view(np.uint64), exp_sig, what + " sigma")
    rel = np.abs(dl.astype(np.float64) - exp_dl)
    bad = rel > 1e-4 * np.abs(exp_dl) + 1e-6
    assert not bad.any(), "%s delta: %d outside tolerance, first at %d" % (what, bad.sum(), np.argmax(bad))


# ---- R-MAT 22: the benchmark step ------------------------------------------------------
def test_rmat22_bfs_direction_optimising():
    g, G = big("rmat22"), dev("rmat22")
    src = graphgen.max_degree_vertex(g)
    st = gg.Stats()
    d = G.bfs(src, step_schedules()["bfs"], stats=st).cpu().numpy()
    assert st.push_iterations > 0 and st.pull_iterations > 0
    assert_int_equal(d, ref("rmat22", "bfs", src), "rmat22 BFS")


def test_rmat22_sssp():
    g, G = big("rmat22"), dev("rmat22")
    src = graphgen.max_degree_vertex(g)
    d = G.sssp(src, step_schedules()["sssp"]).cpu().numpy()
    assert_int_equal(d, ref("rmat22", "sssp", src), "rmat22 SSSP")


def test_rmat22_cc():
    G = dev("rmat22")
    lab = G.cc(step_schedules()["cc"]).cpu().numpy()
    assert_int_equal(lab, ref("rmat22", "cc"), "rmat22 CC")


def test_rmat22_pagerank():
    G = dev("rmat22")
    s = step_schedules()["pr"]
    G.prepare_pull_blocking(s.s1.blocking_size)
    got = G.pagerank(s, iters=20).cpu().numpy()
    check_pr(got, ref("rmat22", "pr"))


def test_rmat22_bc():
    g, G = big("rmat22"), dev("rmat22")
    src = graphgen.max_degree_vertex(g)
    sig, dl = G.bc(src, step_schedules()["bc"])
    es, ed = ref("rmat22", "bc", src)
    check_bc(sig.cpu().numpy(), dl.cpu().numpy(), es, ed, "rmat22 BC")


# ---- R-MAT 20: 64 BFS + 16 BC sources in batches ------------------------------------------
@pytest.mark.parametrize("persistent", [True, False])
def test_rmat20_batched_bfs_64(persistent):
    g, G = big("rmat20"), dev("rmat20")
    srcs = graphgen.sample_giant_sources(g, 64, 7)
    st = gg.Stats()
    d = G.bfs_multi(srcs, gg.make_schedule(direction=gg.PULL, fusion=persistent), stats=st).cpu().numpy()
    assert st.fused == int(persistent)
    for i, s in enumerate(srcs):
        assert_int_equal(d[i], ref("rmat20", "bfs", int(s)), "rmat20 batched BFS row %d" % i)


@pytest.mark.parametrize("persistent", [True, False])
def test_rmat20_batched_bc_16(persistent):
    g, G = big("rmat20"), dev("rmat20")
    srcs = graphgen.sample_giant_sources(g, 64, 7)[:16]
    sig, dl = G.bc_multi(srcs, gg.make_schedule(fusion=persistent))
    sig, dl = sig.cpu().numpy(), dl.cpu().numpy()
    for i, s in enumerate(srcs):
        es, ed = ref("rmat20", "bc", int(s))
        check_bc(sig[i], dl[i], es, ed, "rmat20 batched BC row %d" % i)


# ---- 4096^2 grid: fused and unfused loops ---------------------------------------------------
@pytest.mark.parametrize("fused", [True, False])
def test_grid4096_bfs(fused):
    G = dev("grid4096")
    st = gg.Stats()
    d = G.bfs(0, gg.make_schedule(lb="cm", fusion=fused), stats=st).cpu().numpy()
    assert st.fused == int(fused)
    assert_int_equal(d, ref("grid4096", "bfs", 0), "grid4096 BFS")


@pytest.mark.parametrize("fused", [True, False])
def test_grid4096_sssp_delta512(fused):
    G = dev("grid4096")
    st = gg.Stats()
    d = G.sssp(0, gg.make_schedule(lb="cm", delta=512, fusion=fused), stats=st).cpu().numpy()
    assert st.fused == int(fused)
    assert_int_equal(d, ref("grid4096", "sssp", 0), "grid4096 SSSP delta 512")
