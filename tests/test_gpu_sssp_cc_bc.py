"""GPU parity: delta-stepping SSSP distances and CC labels bit-exact against
the oracle (Dijkstra, union-find) for every schedule form; BC path counts
bit-exact and dependencies within relative 1e-4 of the fp64 Brandes oracle."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal, dev_graph, host_graph, oracle_bc, oracle_cc, oracle_sssp, source

pytestmark = pytest.mark.gpu

LBS = ["vp", "wm", "cm", "strict", "twc", "etwc", "edge_only"]
FUSED_LBS = ["vp", "wm", "cm", "etwc", "strict"]
GRAPHS = ["rmat12", "grid64", "star5000", "cliques", "isolated7", "single"]
INF_DELTA = 2**31 - 1


def _sssp(name, sched, src=None):
    src = source(name) if src is None else src
    st = gg.Stats()
    d = dev_graph(name).sssp(src, sched, stats=st).cpu().numpy()
    assert_int_equal(d, oracle_sssp(name, src), "sssp %s" % name)
    return st


@pytest.mark.parametrize("name", GRAPHS)
@pytest.mark.parametrize("lb", LBS)
@pytest.mark.parametrize("delta", [1, 64])
def test_sssp_lb(name, lb, delta):
    _sssp(name, gg.make_schedule(lb=lb, delta=delta))


def _hybrid_blocked(lb, delta, th, N, create, dedup=True):
    return gg.make_schedule(lb=lb, delta=delta, threshold=th,
                            hybrid={"lb": "edge_only", "edge_blocking": 1, "blocking_size": N,
                                    "frontier_creation": create, "dedup_enable": int(dedup)})


HYBRID_BLOCKED = [("strict", 0.01, 1 << 20, gg.CREATE_FUSED, True),
                  ("etwc", 0.05, 777, gg.CREATE_UNFUSED_BOOLMAP, True),
                  ("cm", 0.001, 64, gg.CREATE_UNFUSED_BITMAP, True),
                  ("strict", 0.2, 3, gg.CREATE_FUSED, False)]


@pytest.mark.parametrize("name", GRAPHS + ["rmat14", "path100k"])
@pytest.mark.parametrize("cfg", HYBRID_BLOCKED)
@pytest.mark.parametrize("delta", [64, 4096])
def test_sssp_hybrid_blocked(name, cfg, delta):
    """Sparse rounds with s1's balancer, dense rounds over the EdgeBlocked COO."""
    lb, th, N, create, dedup = cfg
    _sssp(name, _hybrid_blocked(lb, delta, th, N, create, dedup))


@pytest.mark.parametrize("name", ["rmat12", "grid64", "cliques"])
def test_sssp_blocked_every_round(name):
    _sssp(name, gg.make_schedule(lb="edge_only", delta=64, edge_blocking=True, blocking_size=100))


def test_sssp_hybrid_refusals():
    G = dev_graph("rmat12")
    with pytest.raises(gg.GGError) as e:  # hybrid SSSP loops run unfused
        s = _hybrid_blocked("strict", 64, 0.05, 1 << 20, gg.CREATE_FUSED)
        s.s1.kernel_fusion = 1
        G.sssp(source("rmat12"), s)
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    with pytest.raises(gg.GGError) as e:  # EdgeBlocking needs EDGE_ONLY
        G.sssp(source("rmat12"), gg.make_schedule(lb="cm", edge_blocking=True, blocking_size=64))
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE


@pytest.mark.parametrize("delta", [1, 8, 64, 512, INF_DELTA])
@pytest.mark.parametrize("name", ["grid64", "rmat12", "path100k"])
def test_sssp_delta_invariance(delta, name):
    st = _sssp(name, gg.make_schedule(lb="cm", delta=delta))
    assert st.buckets >= 1


@pytest.mark.parametrize("create", [gg.CREATE_UNFUSED_BOOLMAP, gg.CREATE_UNFUSED_BITMAP])
@pytest.mark.parametrize("dedup_type", [gg.DEDUP_BITMAP, gg.DEDUP_BOOLMAP])
def test_sssp_creation_dedup(create, dedup_type):
    _sssp("rmat12", gg.make_schedule(lb="etwc", creation=create, delta=16))
    _sssp("rmat12", gg.make_schedule(lb="etwc", dedup_type=dedup_type, delta=16))
    _sssp("grid64", gg.make_schedule(lb="vp", dedup=False, delta=16))


@pytest.mark.parametrize("lb", FUSED_LBS)
@pytest.mark.parametrize("delta", [1, 8, 64, 512, INF_DELTA])
@pytest.mark.parametrize("name", ["grid64", "rmat12", "path100k", "star5000", "single", "cliques"])
def test_sssp_fused(lb, delta, name):
    st = _sssp(name, gg.make_schedule(lb=lb, delta=delta, fusion=True))
    assert st.fused == 1


def test_sssp_fused_matches_unfused_bucket_count():
    a = _sssp("grid64", gg.make_schedule(lb="vp", delta=32, fusion=True))
    b = _sssp("grid64", gg.make_schedule(lb="vp", delta=32))
    assert a.buckets == b.buckets


def test_sssp_overflow_reported():
    g = graphgen.path(4)
    w = np.full(g.m, 999_999_999, dtype=np.uint32)
    G = gg.Graph.from_csr(g.n, g.row_ptr, g.col, w)
    for fused in (False, True):
        with pytest.raises(gg.GGError) as e:
            G.sssp(0, gg.make_schedule(fusion=fused, delta=1 << 20))
        assert e.value.status == gg.ERR_OVERFLOW
    d = G.sssp(1, gg.make_schedule(delta=1 << 20)).cpu().numpy()
    assert list(d) == [999_999_999, 0, 999_999_999, 1_999_999_998]


def test_sssp_needs_weights():
    g = host_graph("rmat12")
    G = gg.Graph.from_csr(g.n, g.row_ptr, g.col)
    with pytest.raises(gg.GGError) as e:
        G.sssp(0)
    assert e.value.status == gg.ERR_INVALID_ARG


# ---- CC ------------------------------------------------------------------------------

@pytest.mark.parametrize("name", GRAPHS + ["rmat14", "path100k"])
@pytest.mark.parametrize("lb", LBS)
def test_cc_lb(name, lb):
    st = gg.Stats()
    lab = dev_graph(name).cc(gg.make_schedule(lb=lb), stats=st).cpu().numpy()
    assert_int_equal(lab, oracle_cc(name), "cc %s" % name)
    assert st.iterations >= 1


@pytest.mark.parametrize("name", GRAPHS + ["rmat14", "path100k"])
@pytest.mark.parametrize("lb", FUSED_LBS)
def test_cc_fused(name, lb):
    st = gg.Stats()
    lab = dev_graph(name).cc(gg.make_schedule(lb=lb, fusion=True), stats=st).cpu().numpy()
    assert_int_equal(lab, oracle_cc(name), "cc fused %s" % name)
    assert st.fused == 1


@pytest.mark.parametrize("name", GRAPHS + ["rmat14", "path100k"])
@pytest.mark.parametrize("frac", [64, 41, 7, 1, 0.5])
def test_cc_edge_blocking(name, frac):
    """EDGE_ONLY over the pair list blocked by destination segment: 64
    segments, a ragged last segment, few segments, one, and a width past n."""
    G = dev_graph(name)
    N = max(1, int(-(-G.n // frac))) if frac >= 1 else 2 * G.n + 1
    if -(-G.n // N) > 64:
        N = -(-G.n // 64)
    st = gg.Stats()
    lab = G.cc(gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=N), stats=st).cpu().numpy()
    assert_int_equal(lab, oracle_cc(name), "cc blocked N=%d %s" % (N, name))
    # the blocked list is cached per width: a second run reuses it, same labels
    lab2 = G.cc(gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=N)).cpu().numpy()
    assert np.array_equal(lab, lab2)


def test_cc_edge_blocking_refusals():
    G = dev_graph("rmat12")
    with pytest.raises(gg.GGError) as e:  # 4096 segments
        G.cc(gg.make_schedule(lb="edge_only", edge_blocking=True, blocking_size=1))
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    with pytest.raises(gg.GGError) as e:  # blocking needs the EDGE_ONLY sweep
        G.cc(gg.make_schedule(lb="cm", edge_blocking=True, blocking_size=1024))
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    # the graph still answers afterwards
    assert_int_equal(G.cc(gg.make_schedule(lb="edge_only")).cpu().numpy(), oracle_cc("rmat12"), "cc rmat12")


# ---- BC ------------------------------------------------------------------------------

BC_GRAPHS = ["rmat12", "rmat14", "star5000", "cliques", "isolated7", "single", "fullgrid34", "path100k"]


def _bc(name, sched, src=None):
    src = source(name) if src is None else src
    sigma, delta = dev_graph(name).bc(src, sched)
    es, ed = oracle_bc(name, src)
    assert_int_equal(sigma.cpu().numpy().view(np.uint64), es, "bc sigma %s" % name)
    d = delta.cpu().numpy().astype(np.float64)
    err = np.abs(d - ed)
    assert (err <= 1e-4 * np.abs(ed) + 1e-6).all(), "bc delta %s max err %g" % (name, err.max())
    return delta


@pytest.mark.parametrize("name", BC_GRAPHS)
@pytest.mark.parametrize("lb", LBS)
def test_bc_push_lb(name, lb):
    _bc(name, gg.make_schedule(lb=lb))


@pytest.mark.parametrize("name", BC_GRAPHS)
@pytest.mark.parametrize("rep", [gg.REP_BOOLMAP, gg.REP_BITMAP])
def test_bc_pull_and_hybrid(name, rep):
    _bc(name, gg.make_schedule(direction=gg.PULL, pull_rep=rep))
    s = gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)
    s.s2.pull_rep = rep
    s.threshold = 0.01
    _bc(name, s)


def test_bc_deterministic_and_schedule_invariant_delta():
    a = _bc("rmat14", gg.make_schedule(lb="vp")).cpu().numpy()
    b = _bc("rmat14", gg.make_schedule(lb="etwc")).cpu().numpy()
    c = _bc("rmat14", gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW)).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


def test_bc_sigma_overflow_reported():
    g = graphgen.full_grid(35, 35)
    G = gg.Graph.from_csr(g.n, g.row_ptr, g.col)
    with pytest.raises(gg.GGError) as e:
        G.bc(0)
    assert e.value.status == gg.ERR_OVERFLOW
