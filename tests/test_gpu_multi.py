"""GPU parity for the batched multi-source forms: every row of gg_bfs_multi /
gg_sssp_multi / gg_bc_multi is bit-identical to the single-source call with
the same source (and therefore to the oracle for the integer outputs)."""
import numpy as np
import pytest

import graphgen
import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal, dev_graph, host_graph, oracle_bc, oracle_bfs, oracle_sssp

pytestmark = pytest.mark.gpu


def _sources(name, k, seed=7):
    g = host_graph(name)
    s = graphgen.sample_sources(g, k, seed)
    if s.size < k:  # tiny graphs: repeat and include isolated vertices
        s = np.resize(np.arange(g.n, dtype=np.int32), k)
    return s


def _ms_sched(form):
    if form == "push":
        return gg.make_schedule()
    if form == "pull":
        return gg.make_schedule(direction=gg.PULL)
    if form == "pull_fused":
        return gg.make_schedule(direction=gg.PULL, fusion=True)
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    s.threshold = 0.01
    return s


@pytest.mark.parametrize("name", ["rmat12", "rmat14", "grid64", "star5000", "cliques", "isolated7", "single",
                                  "path100k"])
@pytest.mark.parametrize("k", [1, 7, 64])
@pytest.mark.parametrize("form", ["push", "pull", "hybrid", "pull_fused"])
def test_bfs_multi_matches_single_and_oracle(name, k, form):
    G = dev_graph(name)
    srcs = _sources(name, k)
    st = gg.Stats()
    d = G.bfs_multi(srcs, _ms_sched(form), stats=st).cpu().numpy()
    assert d.shape == (k, host_graph(name).n)
    assert st.fused == (1 if form in ("push", "pull_fused") else 0)
    for i, s in enumerate(srcs):
        assert_int_equal(d[i], oracle_bfs(name, int(s)), "bfs_multi row %d" % i)
    single = G.bfs(int(srcs[0]), gg.make_schedule(lb="etwc")).cpu().numpy()
    assert np.array_equal(d[0], single)


@pytest.mark.parametrize("form", ["push", "pull"])
def test_bfs_multi_duplicate_sources(form):
    G = dev_graph("rmat12")
    s = [5, 5, 9, 5]
    d = G.bfs_multi(s, _ms_sched(form)).cpu().numpy()
    assert np.array_equal(d[0], d[1]) and np.array_equal(d[0], d[3])
    assert_int_equal(d[2], oracle_bfs("rmat12", 9))
    assert_int_equal(d[0], oracle_bfs("rmat12", 5))


@pytest.mark.parametrize("name", ["rmat12", "rmat14", "star5000", "cliques", "isolated7", "single", "fullgrid34",
                                  "path100k"])
@pytest.mark.parametrize("k", [1, 5, 16, 20])
@pytest.mark.parametrize("fused", [False, True])
def test_bc_multi_bit_identical_to_single(name, k, fused):
    G = dev_graph(name)
    srcs = _sources(name, k, seed=11)
    st = gg.Stats()
    sig, dl = G.bc_multi(srcs, gg.make_schedule(fusion=fused), stats=st)
    assert st.fused == (1 if fused else 0)
    sig = sig.cpu().numpy().view(np.uint64)
    dl = dl.cpu().numpy()
    for i, s in enumerate(srcs):
        s1, d1 = G.bc(int(s), gg.make_schedule(lb="etwc"))
        assert np.array_equal(sig[i], s1.cpu().numpy().view(np.uint64)), "sigma row %d" % i
        assert np.array_equal(dl[i].view(np.uint32), d1.cpu().numpy().view(np.uint32)), "delta row %d" % i
        es, ed = oracle_bc(name, int(s))
        assert_int_equal(sig[i], es, "sigma vs oracle row %d" % i)
        err = np.abs(dl[i].astype(np.float64) - ed)
        assert (err <= 1e-4 * np.abs(ed) + 1e-6).all()


@pytest.mark.parametrize("name", ["rmat12", "rmat14", "grid64", "star5000", "cliques", "isolated7", "single",
                                  "path100k", "fullgrid34"])
@pytest.mark.parametrize("k,delta", [(1, 64), (9, 1), (33, 16), (64, 512)])
def test_sssp_multi_matches_oracle(name, k, delta):
    G = dev_graph(name)
    srcs = _sources(name, k, seed=13)
    st = gg.Stats()
    d = G.sssp_multi(srcs, gg.make_schedule(delta=delta), stats=st).cpu().numpy()
    assert d.shape == (k, host_graph(name).n)
    for i, s in enumerate(srcs):
        assert_int_equal(d[i], oracle_sssp(name, int(s)), "sssp_multi row %d (delta %d)" % (i, delta))
    assert st.fused == 1 and st.buckets >= 1
    single = G.sssp(int(srcs[-1]), gg.make_schedule(lb="cm", delta=delta)).cpu().numpy()
    assert np.array_equal(d[-1], single)


def test_sssp_multi_duplicate_sources_and_empty():
    G = dev_graph("grid64")
    d = G.sssp_multi([0, 77, 0, 4095, 77], gg.make_schedule(delta=8)).cpu().numpy()
    assert np.array_equal(d[0], d[2]) and np.array_equal(d[1], d[4])
    for i, s in enumerate([0, 77, 4095]):
        assert_int_equal(d[[0, 1, 3][i]], oracle_sssp("grid64", s))
    assert G.sssp_multi([]).shape == (0, G.n)


def test_sssp_multi_overflow_and_weights():
    g = graphgen.path(4)
    w = np.full(g.m, 999_999_999, dtype=np.uint32)
    G = gg.Graph.from_csr(g.n, g.row_ptr, g.col, w)
    with pytest.raises(gg.GGError) as e:
        G.sssp_multi([1, 0], gg.make_schedule(delta=1 << 20))
    assert e.value.status == gg.ERR_OVERFLOW
    d = G.sssp_multi([1, 2], gg.make_schedule(delta=1 << 20)).cpu().numpy()
    assert list(d[0]) == [999_999_999, 0, 999_999_999, 1_999_999_998]
    assert list(d[1]) == [1_999_999_998, 999_999_999, 0, 999_999_999]
    h = host_graph("rmat12")
    G2 = gg.Graph.from_csr(h.n, h.row_ptr, h.col)
    with pytest.raises(gg.GGError) as e:
        G2.sssp_multi([0])
    assert e.value.status == gg.ERR_INVALID_ARG


def test_multi_argument_errors():
    G = dev_graph("rmat12")
    with pytest.raises(gg.GGError) as e:
        G.bfs_multi(list(range(65)))
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        G.bc_multi([0, G.n])
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        G.sssp_multi([-1])
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        G.sssp_multi([0], gg.make_schedule(delta=0))
    assert e.value.status in (gg.ERR_INVALID_ARG, gg.ERR_UNSUPPORTED_SCHEDULE)


@pytest.mark.parametrize("fused", [False, True])
def test_bc_multi_overflow(fused):
    g = graphgen.full_grid(35, 35)
    G = gg.Graph.from_csr(g.n, g.row_ptr, g.col)
    with pytest.raises(gg.GGError) as e:
        G.bc_multi([0, 1], gg.make_schedule(fusion=fused))
    assert e.value.status == gg.ERR_OVERFLOW
