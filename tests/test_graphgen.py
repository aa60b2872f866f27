"""Input generator checks: sizes, symmetry, determinism (CPU)."""
import numpy as np
import pytest

import graphgen
import oracle


def test_rmat_raw_edge_count_and_determinism():
    s1, d1 = graphgen.rmat_edges(10, 16, seed=5)
    s2, d2 = graphgen.rmat_edges(10, 16, seed=5)
    assert s1.size == 16 * 1024
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    s3, _ = graphgen.rmat_edges(10, 16, seed=6)
    assert not np.array_equal(s1, s3)
    assert s1.min() >= 0 and s1.max() < 1024


def test_rmat_quadrant_probabilities():
    # before the permutation the top bit of (u, v) follows (a, b, c, d)
    src, dst = graphgen.rmat_edges(1, 200000, seed=3)
    # scale 1: vertex ids 0/1 permuted; compare multiset of the four quadrants
    pairs = src.astype(np.int64) * 2 + dst
    counts = np.bincount(pairs, minlength=4) / pairs.size
    perm = graphgen.permutation(2, 4)
    expect = np.zeros(4)
    for (bu, bv), p in {(0, 0): .57, (0, 1): .19, (1, 0): .19, (1, 1): .05}.items():
        expect[perm[bu] * 2 + perm[bv]] = p
    assert np.allclose(counts, expect, atol=0.01)


def test_csr_clean_symmetric_sorted():
    g = graphgen.rmat(12)
    assert oracle.check_csr(g.n, g.row_ptr, g.col) == 0
    assert g.m % 2 == 0
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.m


def test_from_edges_removes_loops_and_duplicates():
    g = graphgen.from_edges(4, [0, 0, 1, 2, 2, 3], [1, 1, 0, 2, 3, 2])
    assert list(g.row_ptr) == [0, 1, 2, 3, 4]
    assert list(g.col) == [1, 0, 3, 2]


def test_grid_counts_and_connectivity():
    W = 64
    g = graphgen.grid(W)
    U = 2 * W * (W - 1)
    D = int(round(0.1 * U))
    assert g.m == 2 * (U - D)
    assert oracle.check_csr(g.n, g.row_ptr, g.col) == 0
    # spanning tree kept: one component
    assert (oracle.cc(g.n, g.row_ptr, g.col) == 0).all()
    assert g.w.min() >= 1 and g.w.max() <= 999


def test_grid_2048_directed_count():
    g = graphgen.grid(2048)
    assert g.m == 15092122


def test_weights_symmetric():
    g = graphgen.rmat(10, weights=True)
    for v in range(0, g.n, 37):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            u = g.col[e]
            lo, hi = g.row_ptr[u], g.row_ptr[u + 1]
            j = lo + np.searchsorted(g.col[lo:hi], v)
            assert g.w[j] == g.w[e]


def test_sources():
    g = graphgen.rmat(12)
    s = graphgen.max_degree_vertex(g)
    deg = g.degrees()
    assert deg[s] == deg.max() and (deg[:s] < deg[s]).all()
    ks = graphgen.sample_sources(g, 64, 7)
    assert len(set(ks.tolist())) == 64 and (deg[ks] > 0).all()
    assert np.array_equal(ks, graphgen.sample_sources(g, 64, 7))


def test_giant_component_sources():
    g = graphgen.disjoint_cliques([3, 40, 5])
    comp = graphgen.giant_component(g)
    assert list(comp) == list(range(3, 43))
    ks = graphgen.sample_giant_sources(g, 10, 7)
    assert len(set(ks.tolist())) == 10 and ((ks >= 3) & (ks < 43)).all()
    assert np.array_equal(ks, graphgen.sample_giant_sources(g, 10, 7))
    h = graphgen.rmat(12)
    lab = oracle.cc(h.n, h.row_ptr, h.col)
    vals, counts = np.unique(lab, return_counts=True)
    big = vals[np.argmax(counts)]
    assert np.array_equal(graphgen.giant_component(h), np.nonzero(lab == big)[0])
