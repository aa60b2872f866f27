"""Shared helpers for the GPU parity tests: cached inputs and oracle results."""
import functools

import numpy as np
import pytest

import graphgen
import oracle

try:
    import torch
    HAS_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAS_GPU = False

needs_gpu = pytest.mark.skipif(not HAS_GPU, reason="needs a GPU")


@functools.lru_cache(maxsize=None)
def host_graph(name: str):
    """Named seeded test inputs (symmetric CSR, some weighted), each
    re-validated by the oracle's CSR check before any result is compared."""
    g = _build_graph(name)
    code = oracle.check_csr(g.n, g.row_ptr, g.col)
    assert code == 0, "input %s fails the oracle's CSR check (code %d)" % (name, code)
    if g.w is not None:
        assert g.w.size == g.m and (g.w.size == 0 or int(g.w.min()) >= 1)
    return g


def _build_graph(name: str):
    if name.startswith("rmat"):
        return graphgen.rmat(int(name[4:]), weights=True)
    if name.startswith("grid"):
        return graphgen.grid(int(name[4:]))
    if name == "star5000":
        g = graphgen.star(5000)
        return graphgen.add_weights(g, 3)
    if name == "path100k":
        g = graphgen.path(100_000)
        return graphgen.add_weights(g, 4)
    if name == "isolated7":
        g = graphgen.isolated(7)
        return graphgen.add_weights(g, 5)
    if name == "single":
        g = graphgen.isolated(1)
        return graphgen.add_weights(g, 6)
    if name == "cliques":
        g = graphgen.disjoint_cliques([1, 3, 70, 300, 2])
        return graphgen.add_weights(g, 7)
    if name == "fullgrid34":
        return graphgen.add_weights(graphgen.full_grid(34, 34), 8)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def dev_graph(name: str):
    import paper_2012_07990_amd as gg
    g = host_graph(name)
    return gg.Graph.from_graphgen(g, validate=True)


def source(name: str) -> int:
    return graphgen.max_degree_vertex(host_graph(name))


@functools.lru_cache(maxsize=None)
def oracle_bfs(name: str, src: int):
    g = host_graph(name)
    return oracle.bfs(g.n, g.row_ptr, g.col, src)


@functools.lru_cache(maxsize=None)
def oracle_sssp(name: str, src: int):
    g = host_graph(name)
    return oracle.sssp(g.n, g.row_ptr, g.col, g.w, src)


@functools.lru_cache(maxsize=None)
def oracle_cc(name: str):
    g = host_graph(name)
    return oracle.cc(g.n, g.row_ptr, g.col)


@functools.lru_cache(maxsize=None)
def oracle_pr(name: str, dangling: bool = True):
    g = host_graph(name)
    return oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20, dangling)


@functools.lru_cache(maxsize=None)
def oracle_bc(name: str, src: int):
    g = host_graph(name)
    return oracle.bc(g.n, g.row_ptr, g.col, src)


def assert_int_equal(got, exp, what=""):
    got = np.asarray(got)
    exp = np.asarray(exp)
    if not np.array_equal(got, exp):
        bad = np.nonzero(got != exp)[0]
        raise AssertionError("%s: %d mismatches, first at %d: got %s expected %s"
                             % (what, bad.size, bad[0], got[bad[0]], exp[bad[0]]))
