"""Pins for the oracle's Brandes BC and EdgeBlocking preprocessing (CPU)."""
import itertools
from math import comb

import numpy as np
import pytest

import graphgen
import oracle
from small_graphs import all_graphs5, dense_adj


def _shortest_paths_by_enumeration(A, s):
    """All shortest s-t paths of a tiny graph, by listing every simple path."""
    n = A.shape[0]
    paths = {}
    for k in range(0, n):
        for mid in itertools.permutations([v for v in range(n) if v != s], k):
            seq = (s,) + mid
            if all(A[seq[i], seq[i + 1]] for i in range(len(seq) - 1)):
                paths.setdefault(seq[-1], []).append(seq)
    out = {}
    for t, ps in paths.items():
        L = min(len(p) for p in ps)
        out[t] = [p for p in ps if len(p) == L]
    return out


def test_bc_exhaustive_5_vertices_by_path_enumeration():
    for mask, g in all_graphs5():
        A = dense_adj(g)
        for s in range(5):
            sp_ = _shortest_paths_by_enumeration(A, s)
            sigma_exp = np.zeros(5, dtype=np.uint64)
            delta_exp = np.zeros(5)
            for t, ps in sp_.items():
                sigma_exp[t] = len(ps)
                if t == s:
                    continue
                for v in range(5):
                    if v in (s, t):
                        continue
                    delta_exp[v] += sum(v in p for p in ps) / len(ps)
            sigma, delta = oracle.bc(g.n, g.row_ptr, g.col, s)
            assert np.array_equal(sigma, sigma_exp), (mask, s)
            assert np.allclose(delta, delta_exp, rtol=1e-14, atol=1e-14), (mask, s)


def _all_source_bc(g):
    tot = np.zeros(g.n)
    for s in range(g.n):
        tot += oracle.bc(g.n, g.row_ptr, g.col, s)[1]
    return tot


@pytest.mark.parametrize("n", [2, 5, 12])
def test_bc_path_closed_forms(n):
    g = graphgen.path(n)
    sigma, delta = oracle.bc(g.n, g.row_ptr, g.col, 0)
    assert (sigma == 1).all()
    i = np.arange(n)
    exp = np.where(i == 0, 0, n - 1 - i).astype(float)
    assert np.array_equal(delta, exp)
    assert np.array_equal(_all_source_bc(g), 2.0 * i * (n - 1 - i))


def test_bc_star_closed_forms():
    k = 6
    g = graphgen.star(k)
    sigma, delta = oracle.bc(g.n, g.row_ptr, g.col, 3)
    assert delta[0] == k - 1 and (np.delete(delta, 0) == 0).all()
    tot = _all_source_bc(g)
    assert tot[0] == k * (k - 1) and (tot[1:] == 0).all()


def test_bc_complete_and_cycle():
    g = graphgen.complete(6)
    assert (_all_source_bc(g) == 0).all()
    c = graphgen.cycle(9)
    t = _all_source_bc(c)
    assert np.allclose(t, t[0], rtol=1e-14)


def test_bc_grid_sigma_binomial_exact():
    W = 34  # max r + c = 66: C(66, 33) ~ 7.2e18 fits uint64
    g = graphgen.full_grid(W, W)
    sigma, _ = oracle.bc(g.n, g.row_ptr, g.col, 0)
    for r in range(W):
        for c in range(W):
            assert int(sigma[r * W + c]) == comb(r + c, r)


def test_bc_grid_sigma_overflow_flagged():
    g = graphgen.full_grid(35, 35)  # r + c = 68: C(68, 34) > 2^64
    with pytest.raises(oracle.OracleOverflow):
        oracle.bc(g.n, g.row_ptr, g.col, 0)


# ---- EdgeBlocking preprocessing ------------------------------------------------

@pytest.mark.parametrize("N", [1, 3, 64, 1000, 1 << 20])
def test_edgeblock_is_stable_sort_by_segment(N):
    g = graphgen.rmat(10)
    src = np.repeat(np.arange(g.n, dtype=np.int32), g.degrees())
    dst = g.col
    os_, od, seg = oracle.edgeblock(g.n, src, dst, N)
    key = dst // N
    order = np.argsort(key, kind="stable")
    assert np.array_equal(os_, src[order]) and np.array_equal(od, dst[order])
    S = (g.n + N - 1) // N
    cnt = np.bincount(key, minlength=S)
    assert seg.size == S + 1 and seg[0] == 0 and seg[-1] == g.m
    assert np.array_equal(np.diff(seg), cnt)
    for s in range(S):
        blk = od[seg[s]:seg[s + 1]]
        assert ((blk >= s * N) & (blk < (s + 1) * N)).all()
        assert (np.diff(os_[seg[s]:seg[s + 1]]) >= 0).all()  # src ascending within a segment


def test_edgeblock_empty():
    os_, od, seg = oracle.edgeblock(10, np.zeros(0, np.int32), np.zeros(0, np.int32), 4)
    assert os_.size == 0 and list(seg) == [0, 0, 0, 0]
