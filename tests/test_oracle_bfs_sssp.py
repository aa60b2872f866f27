"""Pins for the oracle's BFS and SSSP (CPU): brute force, closed forms,
library routines and invariants -- none of them re-runs the oracle's code."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, dijkstra

import graphgen
import oracle
from small_graphs import all_graphs5, floyd_warshall, seeded_weights

INT32_MAX = 2**31 - 1


def test_bfs_exhaustive_5_vertices():
    for mask, g in all_graphs5():
        D = floyd_warshall(g)
        for s in range(5):
            d = oracle.bfs(g.n, g.row_ptr, g.col, s)
            exp = np.where(np.isinf(D[s]), -1, D[s]).astype(np.int32)
            assert np.array_equal(d, exp), (mask, s)


@pytest.mark.parametrize("n", [1, 2, 7, 100])
def test_bfs_path(n):
    g = graphgen.path(n)
    assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col, 0), np.arange(n))


def test_bfs_star_and_complete():
    g = graphgen.star(9)
    assert list(oracle.bfs(g.n, g.row_ptr, g.col, 0)) == [0] + [1] * 9
    assert list(oracle.bfs(g.n, g.row_ptr, g.col, 3)) == [1, 2, 2, 0] + [2] * 6
    k = graphgen.complete(6)
    assert list(oracle.bfs(k.n, k.row_ptr, k.col, 2)) == [1, 1, 0, 1, 1, 1]


def test_bfs_full_grid_manhattan():
    W, H = 13, 7
    g = graphgen.full_grid(W, H)
    d = oracle.bfs(g.n, g.row_ptr, g.col, 0).reshape(H, W)
    r, c = np.mgrid[0:H, 0:W]
    assert np.array_equal(d, r + c)


def test_bfs_isolated_source():
    g = graphgen.isolated(5)
    assert list(oracle.bfs(g.n, g.row_ptr, g.col, 2)) == [-1, -1, 0, -1, -1]


def test_bfs_invariants_rmat():
    g = graphgen.rmat(13)
    s = graphgen.max_degree_vertex(g)
    d = oracle.bfs(g.n, g.row_ptr, g.col, s)
    assert d[s] == 0
    src = np.repeat(np.arange(g.n), g.degrees())
    du, dv = d[src], d[g.col]
    both = (du >= 0) & (dv >= 0)
    assert (np.abs(du[both] - dv[both]) <= 1).all()
    assert ((du >= 0) == (dv >= 0)).all()  # reached set is closed under edges
    # every reached v != s has a neighbour one level up
    has_parent = np.zeros(g.n, bool)
    has_parent[g.col[(du >= 0) & (dv == du + 1)]] = True
    reached = d >= 0
    assert has_parent[reached & (np.arange(g.n) != s)].all()
    # reached set = the component of s (scipy)
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(A, directed=False)
    assert np.array_equal(reached, lab == lab[s])


def test_bfs_matches_scipy_unweighted():
    g = graphgen.rmat(11)
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    for s in [0, 5, graphgen.max_degree_vertex(g)]:
        ref = dijkstra(A, indices=s, unweighted=True)
        exp = np.where(np.isinf(ref), -1, ref).astype(np.int32)
        assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col, s), exp)


def _sssp_expect(D_row):
    return np.where(np.isinf(D_row), INT32_MAX, D_row).astype(np.int64)


def test_sssp_exhaustive_5_vertices():
    for mask, g in all_graphs5():
        w = seeded_weights(g, mask)
        D = floyd_warshall(g, w)
        for s in range(5):
            d = oracle.sssp(g.n, g.row_ptr, g.col, w, s)
            assert np.array_equal(d, _sssp_expect(D[s])), (mask, s)


def test_sssp_random_30():
    for seed in range(20):
        g = graphgen.random_graph(30, 0.12, seed)
        w = seeded_weights(g, seed, wmax=50)
        D = floyd_warshall(g, w)
        for s in (0, 17):
            assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col, w, s), _sssp_expect(D[s]))


def test_sssp_matches_scipy_weighted():
    for g in [graphgen.rmat(11, weights=True), graphgen.grid(64)]:
        A = sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
        ref = dijkstra(A, indices=0)
        assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col, g.w, 0), _sssp_expect(ref))


def test_sssp_unit_weights_equals_bfs_depth_closed_forms():
    g = graphgen.full_grid(9, 11)
    w = np.full(g.m, 7, dtype=np.uint32)
    d = oracle.sssp(g.n, g.row_ptr, g.col, w, 0).reshape(11, 9)
    r, c = np.mgrid[0:11, 0:9]
    assert np.array_equal(d, 7 * (r + c))


def test_sssp_invariants_grid():
    g = graphgen.grid(96)
    d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, 0).astype(np.int64)
    assert d[0] == 0 and (d < INT32_MAX).all()
    src = np.repeat(np.arange(g.n), g.degrees())
    assert (d[g.col] <= d[src] + g.w).all()  # triangle inequality on every edge
    tight = np.zeros(g.n, bool)
    tight[g.col[d[g.col] == d[src] + g.w]] = True
    assert tight[1:].all()  # every vertex but the source has a tight parent


def test_sssp_overflow_flagged():
    g = graphgen.path(4)
    w = np.full(g.m, 999_999_999, dtype=np.uint32)
    with pytest.raises(oracle.OracleOverflow):
        oracle.sssp(g.n, g.row_ptr, g.col, w, 0)
    d = oracle.sssp(g.n, g.row_ptr, g.col, w, 1)  # max 2 hops: 1,999,999,998 fits
    assert list(d) == [999_999_999, 0, 999_999_999, 1_999_999_998]


def test_sssp_unreachable():
    g = graphgen.disjoint_cliques([3, 2])
    w = np.ones(g.m, dtype=np.uint32)
    assert list(oracle.sssp(g.n, g.row_ptr, g.col, w, 4)) == [INT32_MAX] * 3 + [1, 0]
