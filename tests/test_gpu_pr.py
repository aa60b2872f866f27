"""GPU parity: PageRank (FP32) against the fp64 oracle for every traversal
form, and the EdgeBlocked COO against the oracle's preprocessing (bit-exact)."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_07990_amd as gg
from gpu_util import dev_graph, host_graph, oracle_pr

pytestmark = pytest.mark.gpu

FORMS = {
    "pull_vp": dict(lb="vp", direction=gg.PULL),
    "pull_wm": dict(lb="wm", direction=gg.PULL),
    "pull_etwc": dict(lb="etwc", direction=gg.PULL),
    "pull_strict": dict(lb="strict", direction=gg.PULL),
    "push_edge": dict(lb="edge_only", direction=gg.PUSH),
    "push_eb_1k": dict(lb="edge_only", direction=gg.PUSH, edge_blocking=True, blocking_size=1000),
    "push_eb_64": dict(lb="edge_only", direction=gg.PUSH, edge_blocking=True, blocking_size=64),
    "pull_strict_eb_1k": dict(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=1000),
    "pull_strict_eb_64": dict(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=64),
    "pull_strict_eb_big": dict(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=1 << 20),
}
GRAPHS = ["rmat12", "rmat14", "grid64", "star5000", "cliques", "isolated7", "single", "path100k"]


def check_pr(got, exp, dangling=True):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - exp)
    assert err.max() <= 1e-6, "max-abs %g" % err.max()
    assert err.sum() <= 1e-4, "sum-abs %g" % err.sum()
    assert (err / exp).max() <= 1e-3, "max-rel %g" % (err / exp).max()
    if dangling:
        assert abs(got.sum() - 1.0) <= 1e-4


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("name", GRAPHS)
def test_pr_forms(form, name):
    G = dev_graph(name)
    r = G.pagerank(gg.make_schedule(**FORMS[form])).cpu().numpy()
    check_pr(r, oracle_pr(name))


@pytest.mark.parametrize("form", ["pull_vp", "pull_strict", "push_edge"])
def test_pr_no_dangling(form):
    G = dev_graph("rmat12")
    r = G.pagerank(gg.make_schedule(**FORMS[form]), dangling=False).cpu().numpy()
    check_pr(r, oracle_pr("rmat12", False), dangling=False)


@pytest.mark.parametrize("iters", [0, 1, 3])
def test_pr_iteration_counts(iters):
    g = host_graph("rmat12")
    G = dev_graph("rmat12")
    exp = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, iters)
    for form in ("pull_vp", "pull_strict", "push_edge"):
        r = G.pagerank(gg.make_schedule(**FORMS[form]), iters=iters).cpu().numpy()
        check_pr(r, exp)


@pytest.mark.parametrize("form", ["pull_vp", "pull_wm", "pull_etwc", "pull_strict", "pull_strict_eb_1k"])
def test_pr_pull_deterministic(form):
    G = dev_graph("rmat14")
    a = G.pagerank(gg.make_schedule(**FORMS[form])).cpu().numpy()
    b = G.pagerank(gg.make_schedule(**FORMS[form])).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("N", [1, 3, 64, 1000, 1 << 20])
@pytest.mark.parametrize("name", ["rmat12", "grid64", "isolated7"])
def test_edgeblock_layout_matches_oracle(N, name):
    g = host_graph(name)
    G = dev_graph(name)
    G.prepare_edgeblocking(N)
    assert G.prepare_edgeblocking(N) == 0.0  # cached: idempotent
    src, dst, seg = G.edgeblocking_export(N)
    coo_src = np.repeat(np.arange(g.n, dtype=np.int32), g.degrees())
    es, ed, eseg = oracle.edgeblock(g.n, coo_src, g.col, N)
    assert np.array_equal(src.cpu().numpy(), es)
    assert np.array_equal(dst.cpu().numpy(), ed)
    assert np.array_equal(seg, eseg)


@pytest.mark.parametrize("name", ["rmat14", "star5000", "path100k"])
def test_prepare_pull_blocking_then_pagerank(name):
    h = host_graph(name)
    G = gg.Graph.from_graphgen(h)  # a fresh graph: nothing cached yet
    N = 777
    ms = G.prepare_pull_blocking(N)
    assert ms >= 0.0
    assert G.prepare_pull_blocking(N) == 0.0  # cached
    r = G.pagerank(gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=N))
    check_pr(r.cpu().numpy(), oracle_pr(name))
    with pytest.raises(gg.GGError):
        G.prepare_pull_blocking(0)
    G.close()


@pytest.mark.parametrize("N", [0, 3000, 16384, 1 << 20])
@pytest.mark.parametrize("name", ["rmat16", "rmat12", "path100k", "star5000"])
def test_pr_strict_lds_cache_bit_identical(name, N):
    """The STRICT kernel that keeps each segment's highest-degree sources in
    LDS sums the same values in the same order as the one that gathers every
    source from global memory: bit-identical ranks (segments with more and
    with fewer non-isolated vertices than the cache holds, ragged last
    segments, no EdgeBlocking)."""
    G = dev_graph(name)
    kw = dict(lb="strict", direction=gg.PULL)
    if N:
        kw.update(edge_blocking=True, blocking_size=N)
    s = gg.make_schedule(**kw)
    st = gg.Stats()
    st.flags = gg.STATS_TIME_KERNELS
    a = G.pagerank(s, stats=st).cpu().numpy()
    assert b"LDS cache" in bytes(st.kernel_name)
    b = G.pagerank(s, lds_cache=False).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    check_pr(a, oracle_pr(name))


def test_pr_unknown_flags_rejected():
    G = dev_graph("rmat12")
    out = G._empty(G.n, __import__("torch").float32)
    with pytest.raises(gg.GGError) as e:
        gg.gg_pagerank(G, gg.make_schedule(lb="strict", direction=gg.PULL), 0.85, 20, 4, out)
    assert e.value.status == gg.ERR_INVALID_ARG


def test_pr_schedule_errors():
    G = dev_graph("rmat12")
    for kw in [dict(lb="cm", direction=gg.PULL), dict(lb="vp", direction=gg.PUSH),
               dict(lb="vp", direction=gg.PULL, edge_blocking=True),
               dict(lb="strict", direction=gg.PUSH, edge_blocking=True)]:
        with pytest.raises(gg.GGError) as e:
            G.pagerank(gg.make_schedule(**kw))
        assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
