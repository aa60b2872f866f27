"""Exhaustive and closed-form small graphs for the oracle pins (test helper)."""
import itertools

import numpy as np

import graphgen

PAIRS5 = list(itertools.combinations(range(5), 2))  # the 10 possible edges on 5 vertices


def all_graphs5():
    """All 1024 labelled simple graphs on 5 vertices, as (mask, Graph)."""
    for mask in range(1 << len(PAIRS5)):
        es = [PAIRS5[i] for i in range(len(PAIRS5)) if mask >> i & 1]
        s = [a for a, _ in es]
        d = [b for _, b in es]
        yield mask, graphgen.from_edges(5, s, d)


def dense_adj(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    for v in range(g.n):
        A[v, g.col[g.row_ptr[v]:g.row_ptr[v + 1]]] = 1
    return A


def floyd_warshall(g, weights=None):
    """All-pairs shortest path lengths (np.inf when unreachable)."""
    n = g.n
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0)
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            D[v, g.col[e]] = 1 if weights is None else float(weights[e])
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def seeded_weights(g, seed, wmax=9):
    """Symmetric small weights for brute-force checks."""
    w = np.empty(g.m, dtype=np.uint32)
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            a, b = min(v, g.col[e]), max(v, g.col[e])
            w[e] = 1 + graphgen.rng(seed, a * 1000 + b) % wmax
    return w
