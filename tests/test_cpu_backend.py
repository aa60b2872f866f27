"""CPU backend (the library's threaded host implementation, not the oracle)
against the oracle, on the CPU: depths, distances, labels and path counts bit
for bit; PageRank within the FP32-vs-FP64 tolerances and BC dependencies
within relative 1e-4; every result independent of the thread count; error
paths. Runs without a GPU."""
import functools

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_07990_amd as gg


def _inputs(name):
    if name.startswith("drmat"):
        return graphgen.rmat_directed(int(name[5:]), weights=True)
    if name.startswith("rmat"):
        return graphgen.rmat(int(name[4:]), weights=True)
    if name.startswith("grid"):
        return graphgen.grid(int(name[4:]))
    if name == "path2000":
        return graphgen.add_weights(graphgen.path(2000), 3)
    if name == "star3000":
        return graphgen.add_weights(graphgen.star(3000), 4)
    if name == "cliques":
        return graphgen.add_weights(graphgen.disjoint_cliques([1, 3, 70, 300, 2]), 5)
    if name == "isolated7":
        return graphgen.add_weights(graphgen.isolated(7), 6)
    if name == "dgnp200":
        return graphgen.add_weights(graphgen.random_digraph(200, 0.03, 9), 7)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def host(name):
    g = _inputs(name)
    check = oracle.check_digraph if name.startswith("d") else oracle.check_csr
    assert check(g.n, g.row_ptr, g.col) == 0
    return g


@functools.lru_cache(maxsize=None)
def cpu(name):
    return gg.CpuGraph.from_graphgen(host(name), symmetric=not name.startswith("d"), validate=True)


def src_of(name):
    return graphgen.max_degree_vertex(host(name))


SYM = ["rmat12", "rmat14", "grid64", "path2000", "star3000", "cliques", "isolated7"]
ALL = SYM + ["drmat12", "dgnp200"]
THREADS = [1, 3, 8]


@pytest.mark.parametrize("nt", THREADS)
@pytest.mark.parametrize("name", ALL)
def test_cpu_bfs(name, nt):
    g, s = host(name), src_of(name)
    assert np.array_equal(cpu(name).bfs(s, nt), oracle.bfs(g.n, g.row_ptr, g.col, s))


@pytest.mark.parametrize("delta", [1, 64, 4096])
@pytest.mark.parametrize("nt", [1, 8])
@pytest.mark.parametrize("name", ALL)
def test_cpu_sssp(name, nt, delta):
    g, s = host(name), src_of(name)
    assert np.array_equal(cpu(name).sssp(s, delta, nt), oracle.sssp(g.n, g.row_ptr, g.col, g.w, s))


@pytest.mark.parametrize("nt", THREADS)
@pytest.mark.parametrize("name", SYM)
def test_cpu_cc(name, nt):
    g = host(name)
    assert np.array_equal(cpu(name).cc(nt), oracle.cc(g.n, g.row_ptr, g.col))


def _check_pr(got, exp, dangling):
    got = got.astype(np.float64)
    err = np.abs(got - exp)
    assert err.max() <= 1e-6 and err.sum() <= 1e-4 and (err / exp).max() <= 1e-3
    if dangling:
        assert abs(got.sum() - 1.0) <= 1e-4


@pytest.mark.parametrize("dangling", [True, False])
@pytest.mark.parametrize("name", ALL)
def test_cpu_pagerank(name, dangling):
    g = host(name)
    ref = (oracle.pagerank_directed if name.startswith("d") else oracle.pagerank)(
        g.n, g.row_ptr, g.col, 0.85, 20, dangling)
    runs = [cpu(name).pagerank(dangling=dangling, nthreads=nt) for nt in THREADS]
    _check_pr(runs[0], ref, dangling)
    for r in runs[1:]:  # the thread count changes no bit
        assert np.array_equal(r.view(np.int32), runs[0].view(np.int32))


@pytest.mark.parametrize("name", ALL)
def test_cpu_bc(name):
    g, s = host(name), src_of(name)
    try:
        es, ed = oracle.bc(g.n, g.row_ptr, g.col, s)
    except oracle.OracleOverflow:  # path counts past 2^64-1 (the grid): reported, not wrapped
        with pytest.raises(gg.GGError) as e:
            cpu(name).bc(s, 4)
        assert e.value.status == gg.ERR_OVERFLOW
        return
    first = None
    for nt in THREADS:
        sig, dl = cpu(name).bc(s, nt)
        assert np.array_equal(sig, es)
        err = np.abs(dl.astype(np.float64) - ed)
        assert (err <= 1e-4 * np.abs(ed) + 1e-6).all()
        if first is None:
            first = dl
        assert np.array_equal(dl.view(np.int32), first.view(np.int32))


def test_cpu_errors():
    g = host("drmat12")
    with pytest.raises(gg.GGError) as e:
        cpu("drmat12").cc()
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        cpu("rmat12").bfs(-1)
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        cpu("rmat12").sssp(0, 0)
    assert e.value.status == gg.ERR_INVALID_ARG
    unweighted = gg.CpuGraph(g.n, g.row_ptr, g.col, None, symmetric=False)
    with pytest.raises(gg.GGError) as e:
        unweighted.sssp(0)
    assert e.value.status == gg.ERR_INVALID_ARG
    # a distance past INT32_MAX-1 is reported, not wrapped
    p = graphgen.path(4)
    big = gg.CpuGraph(p.n, p.row_ptr, p.col, np.full(p.m, 999_999_999, dtype=np.uint32))
    with pytest.raises(gg.GGError) as e:
        big.sssp(0, 1 << 20)
    assert e.value.status == gg.ERR_OVERFLOW
    assert list(big.sssp(1, 1 << 20)) == [999_999_999, 0, 999_999_999, 1_999_999_998]
    # bad CSR refused when validating
    with pytest.raises(gg.GGError) as e:
        gg.CpuGraph(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 1], np.int32), validate=True)
    assert e.value.status == gg.ERR_INVALID_ARG
