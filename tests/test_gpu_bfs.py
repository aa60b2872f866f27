"""GPU parity: BFS depths through the C ABI are bit-exact against the oracle
for every schedule form (load balance x creation x dedup, push/pull, hybrid,
fused) on seeded inputs spanning several tiles, ragged tails and the
degenerate cases."""
import numpy as np
import pytest

import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal, dev_graph, host_graph, oracle_bfs, source

pytestmark = pytest.mark.gpu

LBS = ["vp", "wm", "cm", "strict", "twc", "etwc", "edge_only"]
CREATES = [gg.CREATE_FUSED, gg.CREATE_UNFUSED_BOOLMAP, gg.CREATE_UNFUSED_BITMAP]
GRAPHS = ["rmat12", "star5000", "grid64", "cliques", "isolated7", "single"]


def _run(name, sched, src=None):
    src = source(name) if src is None else src
    G = dev_graph(name)
    st = gg.Stats()
    d = G.bfs(src, sched, stats=st).cpu().numpy()
    assert_int_equal(d, oracle_bfs(name, src), "bfs %s" % name)
    return st


@pytest.mark.parametrize("name", GRAPHS)
@pytest.mark.parametrize("lb", LBS)
@pytest.mark.parametrize("create", CREATES)
def test_push_lb_creation(name, lb, create):
    _run(name, gg.make_schedule(lb=lb, creation=create))


@pytest.mark.parametrize("dedup_type", [gg.DEDUP_MONOTONIC_COUNTERS, gg.DEDUP_BITMAP, gg.DEDUP_BOOLMAP])
@pytest.mark.parametrize("lb", ["vp", "etwc", "strict"])
def test_push_dedup(dedup_type, lb):
    _run("rmat12", gg.make_schedule(lb=lb, dedup_type=dedup_type))
    _run("rmat12", gg.make_schedule(lb=lb, dedup=False))


@pytest.mark.parametrize("rep", [gg.REP_BOOLMAP, gg.REP_BITMAP])
@pytest.mark.parametrize("create", CREATES)
@pytest.mark.parametrize("name", ["rmat12", "grid64", "star5000"])
def test_pull_only(rep, create, name):
    _run(name, gg.make_schedule(direction=gg.PULL, pull_rep=rep, creation=create))


@pytest.mark.parametrize("threshold", [0.001, 0.01, 0.05, 0.2, 1.0])
@pytest.mark.parametrize("name", ["rmat12", "rmat14"])
def test_hybrid_preset(threshold, name):
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_BFS_HYBRID)
    s.threshold = threshold
    st = _run(name, s)
    assert st.iterations == st.push_iterations + st.pull_iterations


def test_hybrid_switches_direction():
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_BFS_HYBRID)
    s.threshold = 0.01
    st = _run("rmat14", s)
    assert st.push_iterations >= 1 and st.pull_iterations >= 1


@pytest.mark.parametrize("lb", ["vp", "wm", "cm", "etwc", "strict"])
@pytest.mark.parametrize("name", ["rmat12", "rmat14", "grid64", "path100k", "star5000", "single", "cliques",
                                  "isolated7"])
def test_fused(lb, name):
    st = _run(name, gg.make_schedule(lb=lb, fusion=True))
    assert st.fused == 1


@pytest.mark.parametrize("lb", ["vp", "strict"])
@pytest.mark.parametrize("rep", [gg.REP_BOOLMAP, gg.REP_BITMAP])
def test_fused_hybrid(rep, lb):
    s = gg.make_schedule(lb=lb, fusion=True, hybrid={"direction": gg.PULL, "pull_rep": rep, "lb": "vp"},
                         threshold=0.01)
    st = _run("rmat14", s)
    assert st.fused == 1 and st.pull_iterations >= 1


def test_fused_strict_every_source_small_graph():
    g = host_graph("cliques")
    for s in range(g.n):
        _run("cliques", gg.make_schedule(lb="strict", fusion=True), src=s)


def test_every_source_small_graph():
    g = host_graph("cliques")
    for s in range(g.n):
        _run("cliques", gg.make_schedule(lb="etwc"), src=s)


def test_edge_counter_push_vp_counts_reached_degrees():
    name = "rmat12"
    g = host_graph(name)
    src = source(name)
    st = gg.Stats()
    st.flags = gg.STATS_COUNT_EDGES
    G = dev_graph(name)
    G.bfs(src, gg.make_schedule(lb="vp"), stats=st)
    reached = oracle_bfs(name, src) >= 0
    assert st.edges_examined == int(g.degrees()[reached].sum())
    assert st.vertices_processed == int(reached.sum())


def test_bad_source_and_schedule_errors():
    G = dev_graph("rmat12")
    with pytest.raises(gg.GGError) as e:
        G.bfs(-1)
    assert e.value.status == gg.ERR_INVALID_ARG
    s = gg.make_schedule(lb="twc", fusion=True)
    with pytest.raises(gg.GGError) as e:
        G.bfs(0, s)
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    s = gg.make_schedule(lb="etwc", direction=gg.PULL)
    with pytest.raises(gg.GGError) as e:
        G.bfs(0, s)
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
