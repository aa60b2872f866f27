"""Pins for the oracle's CC and PageRank (CPU)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle
from small_graphs import all_graphs5, dense_adj


def _canon_min_label(lab):
    """Relabel components by their smallest member id."""
    out = np.empty_like(lab)
    for c in np.unique(lab):
        idx = np.nonzero(lab == c)[0]
        out[idx] = idx.min()
    return out.astype(np.int32)


def test_cc_exhaustive_transitive_closure():
    for mask, g in all_graphs5():
        R = (dense_adj(g) + np.eye(5, dtype=np.int64)) > 0
        for _ in range(3):
            R = (R.astype(np.int64) @ R.astype(np.int64)) > 0
        exp = np.array([np.nonzero(R[v])[0].min() for v in range(5)], dtype=np.int32)
        assert np.array_equal(oracle.cc(g.n, g.row_ptr, g.col), exp), mask


def test_cc_matches_scipy():
    for g in [graphgen.rmat(13), graphgen.grid(50), graphgen.random_graph(200, 0.006, 3)]:
        A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
        _, lab = connected_components(A, directed=False)
        assert np.array_equal(oracle.cc(g.n, g.row_ptr, g.col), _canon_min_label(lab))


def test_cc_closed_forms():
    g = graphgen.disjoint_cliques([3, 1, 4, 2])
    assert list(oracle.cc(g.n, g.row_ptr, g.col)) == [0, 0, 0, 3, 4, 4, 4, 4, 8, 8]
    g = graphgen.isolated(6)
    assert list(oracle.cc(g.n, g.row_ptr, g.col)) == list(range(6))


def test_cc_invariants_rmat():
    g = graphgen.rmat(12)
    L = oracle.cc(g.n, g.row_ptr, g.col)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert (L[src] == L[g.col]).all()
    assert (L <= np.arange(g.n)).all()
    assert (L[L] == L).all()


# ---- PageRank -----------------------------------------------------------------

def _google_power(g, d, iters, dangling=True):
    """Dense Google-matrix power iteration (n small)."""
    n = g.n
    A = dense_adj(g).astype(np.float64)
    deg = A.sum(axis=0)
    P = np.divide(A, deg[None, :], out=np.zeros_like(A), where=deg[None, :] > 0)
    dmask = (deg == 0).astype(np.float64)
    G = d * P + (d * np.outer(np.ones(n), dmask) / n if dangling else 0.0)
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = G @ x + (1 - d) / n
    return x


def test_pr_dense_google_matrix():
    for seed in range(12):
        g = graphgen.random_graph(40, 0.05, seed)  # sparse: has isolated vertices
        assert (g.degrees() == 0).any() or seed > 0
        for dang in (True, False):
            exp = _google_power(g, 0.85, 20, dang)
            got = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20, dangling=dang)
            assert np.max(np.abs(got - exp)) < 1e-15, (seed, dang)


def test_pr_exhaustive_5_vertices():
    for mask, g in all_graphs5():
        exp = _google_power(g, 0.85, 20)
        assert np.max(np.abs(oracle.pagerank(g.n, g.row_ptr, g.col) - exp)) < 1e-15, mask


def test_pr_regular_graphs_stay_uniform():
    for g in [graphgen.cycle(17), graphgen.complete(9), graphgen.isolated(11)]:
        r = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20)
        assert np.allclose(r, 1.0 / g.n, rtol=1e-14, atol=0)


def test_pr_isolated_without_dangling_mass():
    g = graphgen.isolated(8)
    r = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 3, dangling=False)
    assert np.allclose(r, 0.15 / 8, rtol=1e-15)


def test_pr_star_exact_rational_recurrence():
    k = 7
    N = k + 1
    d = Fraction(85, 100)
    c = l = Fraction(1, N)
    for _ in range(20):
        c, l = (1 - d) / N + d * k * l, (1 - d) / N + d * c / k
    g = graphgen.star(k)
    r = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20)
    assert abs(r[0] - float(c)) <= 1e-15
    assert np.all(np.abs(r[1:] - float(l)) <= 1e-15)


def test_pr_mass_sums_to_one():
    g = graphgen.rmat(12)  # many isolated vertices after cleaning
    assert (g.degrees() == 0).any()
    r = oracle.pagerank(g.n, g.row_ptr, g.col)
    assert abs(r.sum() - 1.0) < 1e-12
    assert (r >= 0.15 / g.n * (1 - 1e-12)).all()
