"""Pins for the oracle on directed graphs (rows are out-edges), on the CPU:
the directed CSR check per defect, directed PageRank against the dense Google
matrix and closed forms, BFS/SSSP against Floyd-Warshall and scipy's directed
Dijkstra, Brandes BC against an enumeration of all shortest paths. None of
them re-runs the oracle's code."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import graphgen
import oracle
from small_graphs import dense_adj, floyd_warshall

INT32_MAX = 2**31 - 1


def _digraphs():
    for n, p, seed in [(5, 0.3, 1), (6, 0.4, 2), (7, 0.25, 3), (8, 0.5, 4), (10, 0.2, 5), (12, 0.15, 6),
                       (30, 0.08, 7), (40, 0.05, 8)]:
        yield graphgen.random_digraph(n, p, seed)


def _dir_weights(g, seed, wmax=9):
    """Small per-entry weights (direction matters: keyed by the ordered pair)."""
    w = np.empty(g.m, dtype=np.uint32)
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            w[e] = 1 + graphgen.rng(seed, v * 1000 + int(g.col[e])) % wmax
    return w


# ---- directed CSR check ------------------------------------------------------------
def test_check_digraph_accepts_non_symmetric_and_names_each_defect():
    rp = np.array([0, 2, 3, 3], dtype=np.int32)
    col = np.array([1, 2, 2], dtype=np.int32)  # 0->1, 0->2, 1->2: not symmetric
    assert oracle.check_digraph(3, rp, col) == 0
    assert oracle.check_csr(3, rp, col) == 6  # the symmetric check refuses it
    assert oracle.check_digraph(3, np.array([1, 2, 3, 3], np.int32), col) == 1      # row_ptr[0] != 0
    assert oracle.check_digraph(3, np.array([0, 2, 1, 3], np.int32), col) == 2      # not monotone
    assert oracle.check_digraph(3, rp, np.array([1, 3, 2], np.int32)) == 3          # out of range
    assert oracle.check_digraph(3, rp, np.array([1, 2, 1], np.int32)) == 4          # self-loop 1->1
    assert oracle.check_digraph(3, rp, np.array([2, 1, 2], np.int32)) == 5          # unsorted row
    assert oracle.check_digraph(3, rp, np.array([1, 1, 2], np.int32)) == 5          # duplicate entry


def test_directed_generators_pass_the_check():
    for g in list(_digraphs()) + [graphgen.rmat_directed(12)]:
        assert oracle.check_digraph(g.n, g.row_ptr, g.col) == 0


def test_rmat_directed_is_the_unmirrored_edge_set():
    g, h = graphgen.rmat_directed(10), graphgen.rmat(10)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    # symmetrising the directed graph gives the symmetric R-MAT
    s = graphgen.from_edges(g.n, src, g.col)
    assert np.array_equal(s.row_ptr, h.row_ptr) and np.array_equal(s.col, h.col)
    assert g.m < h.m


# ---- PageRank -------------------------------------------------------------------------
def _google_power(g, d, iters, dangling):
    """Dense Google-matrix power iteration: r <- (1-d)/n + d (M r + D/n) with
    M[v, u] = 1/outdeg(u) for every edge u -> v."""
    n = g.n
    A = dense_adj(g).astype(np.float64)   # A[u, v] = 1 for u -> v
    out = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = out > 0
    M[:, nz] = (A[nz, :] / out[nz, None]).T
    r = np.full(n, 1.0 / n)
    for _ in range(iters):
        D = r[~nz].sum() if dangling else 0.0
        r = (1 - d) / n + d * (M @ r + D / n)
    return r


@pytest.mark.parametrize("dangling", [True, False])
def test_pagerank_directed_matches_dense_google_matrix(dangling):
    for g in _digraphs():
        for iters in [0, 1, 3, 20]:
            got = oracle.pagerank_directed(g.n, g.row_ptr, g.col, 0.85, iters, dangling)
            exp = _google_power(g, 0.85, iters, dangling)
            assert np.allclose(got, exp, rtol=1e-12, atol=1e-15), (g.name, iters)


def test_pagerank_directed_closed_forms():
    # directed cycle: every vertex passes all its rank on, ranks stay 1/n
    n = 9
    i = np.arange(n)
    c = graphgen.from_edges_directed(n, i, (i + 1) % n)
    assert np.allclose(oracle.pagerank_directed(c.n, c.row_ptr, c.col, 0.85, 20), 1.0 / n, rtol=1e-14)
    # in-star: k leaves point at the centre 0, which has no out-edge (the
    # only dangling vertex); by symmetry every leaf has the same rank, so the
    # ranks follow a two-value recurrence: centre <- (1-d)/n + d (k leaf +
    # centre/n), leaf <- (1-d)/n + d centre/n
    k = 5
    s = graphgen.from_edges_directed(k + 1, np.arange(1, k + 1), np.zeros(k, dtype=np.int64))
    n = k + 1
    d = 0.85
    rc, rl = 1.0 / n, 1.0 / n
    for _ in range(7):
        rc, rl = (1 - d) / n + d * (k * rl + rc / n), (1 - d) / n + d * (rc / n)
    got = oracle.pagerank_directed(s.n, s.row_ptr, s.col, d, 7)
    assert abs(got[0] - rc) < 1e-15 and np.allclose(got[1:], rl, rtol=1e-14)
    # variant 0 keeps the total mass at 1
    for g in _digraphs():
        assert abs(oracle.pagerank_directed(g.n, g.row_ptr, g.col, 0.85, 20).sum() - 1.0) < 1e-12


def test_pagerank_directed_on_symmetric_graph_equals_pagerank():
    g = graphgen.rmat(9)
    a = oracle.pagerank_directed(g.n, g.row_ptr, g.col, 0.85, 20)
    b = oracle.pagerank(g.n, g.row_ptr, g.col, 0.85, 20)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-16)


# ---- BFS / SSSP on directed graphs ------------------------------------------------------
def test_directed_bfs_and_sssp_against_floyd_warshall():
    for g in _digraphs():
        D = floyd_warshall(g)
        w = _dir_weights(g, 11)
        Dw = floyd_warshall(g, w)
        for s in range(g.n):
            exp = np.where(np.isinf(D[s]), -1, D[s]).astype(np.int32)
            assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col, s), exp), (g.name, s)
            expw = np.where(np.isinf(Dw[s]), INT32_MAX, Dw[s]).astype(np.int64)
            assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col, w, s).astype(np.int64), expw), (g.name, s)


def test_directed_sssp_against_scipy_on_rmat():
    g = graphgen.rmat_directed(11, weights=True)
    A = sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    for s in [graphgen.max_degree_vertex(g), 0, 17]:
        exp = dijkstra(A, directed=True, indices=s)
        exp = np.where(np.isinf(exp), INT32_MAX, exp).astype(np.int64)
        got = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s).astype(np.int64)
        assert np.array_equal(got, exp)
        hops = dijkstra(sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n)), directed=True,
                        indices=s)
        assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col, s), np.where(np.isinf(hops), -1, hops).astype(np.int32))


# ---- BC on directed graphs ------------------------------------------------------------------
def _directed_shortest_paths(A, s):
    n = A.shape[0]
    paths = {}
    for k in range(0, n):
        for mid in itertools.permutations([v for v in range(n) if v != s], k):
            seq = (s,) + mid
            if all(A[seq[i], seq[i + 1]] for i in range(len(seq) - 1)):
                paths.setdefault(seq[-1], []).append(seq)
    return {t: [p for p in ps if len(p) == min(len(q) for q in ps)] for t, ps in paths.items()}


def test_directed_bc_by_path_enumeration():
    for n, p, seed in [(5, 0.4, 21), (6, 0.35, 22), (6, 0.5, 23), (7, 0.3, 24)]:
        g = graphgen.random_digraph(n, p, seed)
        A = dense_adj(g)
        for s in range(n):
            sp_ = _directed_shortest_paths(A, s)
            sigma_exp = np.zeros(n, dtype=np.uint64)
            delta_exp = np.zeros(n)
            for t, ps in sp_.items():
                sigma_exp[t] = len(ps)
                if t == s:
                    continue
                for v in range(n):
                    if v not in (s, t):
                        delta_exp[v] += sum(v in q for q in ps) / len(ps)
            sigma, delta = oracle.bc(g.n, g.row_ptr, g.col, s)
            assert np.array_equal(sigma, sigma_exp), (n, seed, s)
            assert np.allclose(delta, delta_exp, rtol=1e-14, atol=1e-14), (n, seed, s)
