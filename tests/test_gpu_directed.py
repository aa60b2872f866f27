"""GPU parity on directed graphs (CSR rows are out-edges, no GG_SYMMETRIC):
BFS depths, SSSP distances and BC path counts bit for bit, BC dependencies
within relative 1e-4 and PageRank within the FP32-vs-FP64 tolerances, against
the oracle's directed definitions. PULL steps read the graph's transpose
(built by the library on first use); PUSH steps follow out-edges."""
import functools

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal

pytestmark = pytest.mark.gpu


def _inputs(name):
    if name.startswith("drmat"):
        return graphgen.rmat_directed(int(name[5:]), weights=True)
    if name == "dgnp300":
        return graphgen.add_weights(graphgen.random_digraph(300, 0.02, 41), 42)
    if name == "dchain":  # 0 -> 1 -> ... -> 4999: one vertex per level, no way back
        i = np.arange(4999)
        return graphgen.add_weights(graphgen.from_edges_directed(5000, i, i + 1), 43)
    if name == "instar":  # 3000 leaves -> centre 0: the centre is the only dangling vertex
        k = 3000
        return graphgen.add_weights(graphgen.from_edges_directed(k + 1, np.arange(1, k + 1), np.zeros(k)), 44)
    if name == "outstar":  # centre 0 -> 3000 leaves
        k = 3000
        return graphgen.add_weights(graphgen.from_edges_directed(k + 1, np.zeros(k), np.arange(1, k + 1)), 45)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def host(name):
    g = _inputs(name)
    assert oracle.check_digraph(g.n, g.row_ptr, g.col) == 0
    return g


@functools.lru_cache(maxsize=None)
def dev(name):
    g = host(name)
    return gg.Graph.from_csr(g.n, g.row_ptr, g.col, g.w, symmetric=False, validate=True)


def src_of(name):
    return 0 if name in ("dchain", "outstar", "instar") else graphgen.max_degree_vertex(host(name))


GRAPHS = ["drmat12", "drmat14", "dgnp300", "dchain", "instar", "outstar"]


def _hybrid(lb, th=0.01):
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    s.s1.load_balance = gg.LB_NAMES[lb]
    s.threshold = th
    return s


BFS_SCHEDULES = {
    "push-vp": lambda: gg.make_schedule(lb="vp"),
    "push-strict": lambda: gg.make_schedule(lb="strict"),
    "push-etwc": lambda: gg.make_schedule(lb="etwc"),
    "push-twc": lambda: gg.make_schedule(lb="twc"),
    "push-edge_only": lambda: gg.make_schedule(lb="edge_only"),
    "pull-boolmap": lambda: gg.make_schedule(direction=gg.PULL),
    "pull-bitmap": lambda: gg.make_schedule(direction=gg.PULL, pull_rep=gg.REP_BITMAP,
                                            creation=gg.CREATE_UNFUSED_BITMAP),
    "hybrid-strict": lambda: _hybrid("strict"),
    "hybrid-etwc-0.001": lambda: _hybrid("etwc", 0.001),
    "fused-cm": lambda: gg.make_schedule(lb="cm", fusion=True),
    "fused-hybrid": lambda: gg.make_schedule(lb="vp", fusion=True, threshold=0.01,
                                             hybrid={"direction": gg.PULL, "pull_rep": gg.REP_BITMAP}),
}


@pytest.mark.parametrize("key", sorted(BFS_SCHEDULES))
@pytest.mark.parametrize("name", GRAPHS)
def test_directed_bfs(name, key):
    g, s = host(name), src_of(name)
    d = dev(name).bfs(s, BFS_SCHEDULES[key]()).cpu().numpy()
    assert_int_equal(d, oracle.bfs(g.n, g.row_ptr, g.col, s), "bfs %s %s" % (name, key))


@pytest.mark.parametrize("sched", ["strict-d64", "etwc-d1", "vp-d4096", "fused-cm-d512", "cm-d8"])
@pytest.mark.parametrize("name", GRAPHS)
def test_directed_sssp(name, sched):
    parts = sched.split("-")
    fused = parts[0] == "fused"
    lb = parts[1] if fused else parts[0]
    delta = int(parts[-1][1:])
    g, s = host(name), src_of(name)
    d = dev(name).sssp(s, gg.make_schedule(lb=lb, delta=delta, fusion=fused)).cpu().numpy()
    assert_int_equal(d, oracle.sssp(g.n, g.row_ptr, g.col, g.w, s), "sssp %s %s" % (name, sched))


@pytest.mark.parametrize("name", ["drmat12", "dgnp300", "dchain"])
def test_directed_sssp_hybrid_blocked(name):
    """Dense rounds over the EdgeBlocked COO of the out-edges."""
    g, s = host(name), src_of(name)
    sched = gg.make_schedule(lb="strict", delta=64, threshold=0.01,
                             hybrid={"lb": "edge_only", "edge_blocking": 1, "blocking_size": 1000})
    d = dev(name).sssp(s, sched).cpu().numpy()
    assert_int_equal(d, oracle.sssp(g.n, g.row_ptr, g.col, g.w, s), "sssp hybrid blocked %s" % name)


def test_directed_batched_sssp_matches_single_calls():
    name = "drmat12"
    g = host(name)
    srcs = [int(x) for x in graphgen.sample_sources(g, 8, 5)]
    dm = dev(name).sssp_multi(srcs, gg.make_schedule(delta=64)).cpu().numpy()
    for i, s in enumerate(srcs):
        assert_int_equal(dm[i], oracle.sssp(g.n, g.row_ptr, g.col, g.w, s), "batched sssp %d" % s)


PR_FORMS = {
    "pull_vp": dict(lb="vp", direction=gg.PULL),
    "pull_wm": dict(lb="wm", direction=gg.PULL),
    "pull_etwc": dict(lb="etwc", direction=gg.PULL),
    "pull_strict": dict(lb="strict", direction=gg.PULL),
    "pull_strict_eb_1k": dict(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=1000),
    "pull_strict_eb_4k": dict(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=4096),
    "push_edge": dict(lb="edge_only", direction=gg.PUSH),
    "push_eb_1k": dict(lb="edge_only", direction=gg.PUSH, edge_blocking=True, blocking_size=1000),
}


def check_pr(got, exp, dangling=True):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - exp)
    assert err.max() <= 1e-6, "max-abs %g" % err.max()
    assert err.sum() <= 1e-4, "sum-abs %g" % err.sum()
    assert (err / exp).max() <= 1e-3, "max-rel %g" % (err / exp).max()
    if dangling:
        assert abs(got.sum() - 1.0) <= 1e-4


@pytest.mark.parametrize("dangling", [True, False])
@pytest.mark.parametrize("form", sorted(PR_FORMS))
@pytest.mark.parametrize("name", GRAPHS)
def test_directed_pagerank(name, form, dangling):
    g = host(name)
    r = dev(name).pagerank(gg.make_schedule(**PR_FORMS[form]), dangling=dangling).cpu().numpy()
    check_pr(r, oracle.pagerank_directed(g.n, g.row_ptr, g.col, 0.85, 20, dangling), dangling)


def test_directed_pagerank_lds_cache_bit_identical():
    G = dev("drmat14")
    s = gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=4096)
    a = G.pagerank(s).cpu().numpy()
    b = G.pagerank(s, lds_cache=False).cpu().numpy()
    assert np.array_equal(a.view(np.int32), b.view(np.int32))


@pytest.mark.parametrize("sched", ["push-vp", "push-strict", "pull", "hybrid-strict"])
@pytest.mark.parametrize("name", GRAPHS)
def test_directed_bc(name, sched):
    if sched == "pull":
        s = gg.make_schedule(direction=gg.PULL)
    elif sched.startswith("hybrid"):
        s = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
        s.s1.load_balance = gg.LB_STRICT
        s.threshold = 0.01
    else:
        s = gg.make_schedule(lb=sched.split("-")[1])
    g, src = host(name), src_of(name)
    sig, dl = dev(name).bc(src, s)
    es, ed = oracle.bc(g.n, g.row_ptr, g.col, src)
    assert_int_equal(sig.cpu().numpy().view(np.uint64), es, "bc sigma %s %s" % (name, sched))
    dl = dl.cpu().numpy().astype(np.float64)
    err = np.abs(dl - ed)
    assert (err <= 1e-4 * np.abs(ed) + 1e-6).all(), "bc delta %s max err %g" % (name, err.max())


def test_directed_refusals():
    G = dev("drmat12")
    with pytest.raises(gg.GGError) as e:
        G.cc()
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        G.bfs_multi([0, 1])
    assert e.value.status == gg.ERR_INVALID_ARG
