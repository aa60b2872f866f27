"""Programs in the algorithm and scheduling languages, compiled to HIP by the
library's compiler (modules built by __graft_entry__.build() into
paper_2012_07990_amd/_gen/), run on the GPU and checked against the oracle:
BFS parents form a valid shortest-path tree of the oracle's depths, SSSP
distances and CC labels bit for bit, PageRank (fp64, no dangling term)
within 1e-12 of the oracle. Several schedules per program (unfused loops and
loops generated as one persistent launch), symmetric and directed graphs,
and the errors the generated entry point reports."""
import functools
import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_07990_amd as gg
from paper_2012_07990_amd import compiler

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def module(name):
    so = os.path.join(compiler.GEN_DIR, name + ".so")
    assert os.path.exists(so), "%s missing: run __graft_entry__.build()" % so
    return compiler.load(so, compiler.VARIANTS[name][1])


def _inputs(name):
    if name.startswith("drmat"):
        return graphgen.rmat_directed(int(name[5:]), weights=True)
    if name.startswith("rmat"):
        return graphgen.rmat(int(name[4:]), weights=True)
    if name.startswith("grid"):
        return graphgen.grid(int(name[4:]))
    if name == "cliques":
        return graphgen.add_weights(graphgen.disjoint_cliques([1, 3, 70, 300, 2]), 5)
    if name == "path3000":
        return graphgen.add_weights(graphgen.path(3000), 3)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def host(name):
    return _inputs(name)


@functools.lru_cache(maxsize=None)
def dev(name):
    g = host(name)
    return gg.Graph.from_csr(g.n, g.row_ptr, g.col, g.w, symmetric=not name.startswith("d"), validate=True)


def src_of(name):
    return graphgen.max_degree_vertex(host(name))


SYM = ["rmat12", "rmat14", "grid48", "cliques", "path3000"]


def check_parents(g, parent, src, directed=False):
    depth = oracle.bfs(g.n, g.row_ptr, g.col, src)
    assert parent[src] == src
    reached = depth >= 0
    assert np.array_equal(parent >= 0, reached)
    v = np.flatnonzero(reached & (np.arange(g.n) != src))
    p = parent[v]
    assert (depth[p] == depth[v] - 1).all()
    # p -> v must be an edge (u's out-row holds v)
    rp, col = g.row_ptr, g.col
    for a, b in zip(p, v):
        row = col[rp[a]:rp[a + 1]]
        assert b in row


@pytest.mark.parametrize("variant", ["bfs_push_twce", "bfs_push_strict_boolmap", "bfs_pull_bitmap", "bfs_hybrid",
                                     "bfs_fused_hybrid_strict", "bfs_fused_wm_boolpull"])
@pytest.mark.parametrize("name", SYM + ["drmat12"])
def test_generated_bfs(variant, name):
    g, s = host(name), src_of(name)
    parent = module(variant).run(dev(name), [s])["parent"].cpu().numpy()
    check_parents(g, parent, s)


@pytest.mark.parametrize("variant", ["sssp_push_strict", "sssp_push_vp_nodedup", "sssp_pull", "sssp_fused_etwc",
                                     "sssp_fused_vp_nodedup"])
@pytest.mark.parametrize("name", SYM)
def test_generated_sssp(variant, name):
    g, s = host(name), src_of(name)
    dist = module(variant).run(dev(name), [s])["dist"].cpu().numpy()
    assert np.array_equal(dist, oracle.sssp(g.n, g.row_ptr, g.col, g.w, s))


PQ_VARIANTS = ["sssp_pq_strict_d64", "sssp_pq_etwc_d1", "sssp_pq_cm_d4096_boolmap", "sssp_pq_vp_d512_nodedup"]


@pytest.mark.parametrize("variant", PQ_VARIANTS)
@pytest.mark.parametrize("name", SYM + ["drmat12"])
def test_generated_priority_queue(variant, name):
    """applyUpdatePriority over the delta-stepping buckets configDelta sets."""
    g, s = host(name), src_of(name)
    dist = module(variant).run(dev(name), [s])["dist"].cpu().numpy()
    assert np.array_equal(dist, oracle.sssp(g.n, g.row_ptr, g.col, g.w, s))


@pytest.mark.parametrize("variant", ["sssp_push_strict", "sssp_push_vp_nodedup", "sssp_fused_etwc"])
def test_generated_sssp_directed(variant):
    g, s = host("drmat12"), src_of("drmat12")
    dist = module(variant).run(dev("drmat12"), [s])["dist"].cpu().numpy()
    assert np.array_equal(dist, oracle.sssp(g.n, g.row_ptr, g.col, g.w, s))


@pytest.mark.parametrize("variant", ["cc_push_etwc", "cc_push_edge_only", "cc_fused_cm"])
@pytest.mark.parametrize("name", SYM)
def test_generated_cc(variant, name):
    g = host(name)
    ids = module(variant).run(dev(name))["IDs"].cpu().numpy()
    assert np.array_equal(ids, oracle.cc(g.n, g.row_ptr, g.col))


@pytest.mark.parametrize("variant", ["pagerank_pull", "pagerank_push_strict", "pagerank_push_blocked"])
@pytest.mark.parametrize("name", SYM + ["drmat12"])
def test_generated_pagerank(variant, name):
    g = host(name)
    fn = oracle.pagerank_directed if name.startswith("d") else oracle.pagerank
    ref = fn(g.n, g.row_ptr, g.col, 0.85, 20, False)
    got = module(variant).run(dev(name))["old_rank"].cpu().numpy()
    # fp64 on both sides; only the summation order differs
    assert np.abs(got - ref).max() <= 1e-12


def test_generated_errors():
    m = module("bfs_push_twce")
    G = dev("rmat12")
    for bad in ([-1], [G.n], []):
        with pytest.raises(gg.GGError) as e:
            m.run(G, bad)
        assert e.value.status == gg.ERR_INVALID_ARG
    # a weighted PULL over a directed graph would read in-edge weights in out-edge order: refused
    with pytest.raises(gg.GGError) as e:
        module("sssp_pull").run(dev("drmat12"), [src_of("drmat12")])
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    # an unweighted graph for a weighted program
    h = host("rmat12")
    G2 = gg.Graph.from_csr(h.n, h.row_ptr, h.col, None, symmetric=True)
    with pytest.raises(gg.GGError) as e:
        module("sssp_push_strict").run(G2, [0])
    assert e.value.status == gg.ERR_INVALID_ARG
    # the module still runs after the errors
    check_parents(h, m.run(G, [3])["parent"].cpu().numpy(), 3)


@pytest.mark.parametrize("variant", ["bfs_rounds", "bfs_rounds_fused"])
@pytest.mark.parametrize("name", SYM + ["drmat12"])
def test_generated_loop_statements(variant, name):
    """Scalar statements and a vertex operator inside the frontier loop: run on
    the host around each round, or inside the one persistent kernel with main's
    locals hoisted to device memory; both give the same counts."""
    g, s = host(name), src_of(name)
    out = module(variant).run(dev(name), [s])
    parent = out["parent"].cpu().numpy()
    check_parents(g, parent, s)
    rounds = int(oracle.bfs(g.n, g.row_ptr, g.col, s).max()) + 1  # non-empty frontiers
    info = out["info"].cpu().numpy()
    assert info[0] == rounds and info[1] == 10 + rounds * rounds  # work += 2 * round - 1 each round
    assert (out["seen"].cpu().numpy() == rounds).all()
