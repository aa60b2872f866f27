"""Pins for the oracle's CSR re-validation (CPU).

The oracle re-checks every input graph (rows sorted and duplicate-free,
columns in range, no self-loops, symmetric) so that a graph-builder bug cannot
hide behind matching GPU and oracle results. These tests plant each kind of
defect and require its specific code, and compare the valid/invalid verdict on
random small arrays with a set-based definition written here independently.
"""
import numpy as np
import pytest

import graphgen
import oracle

# codes of oracle_check_csr
OK, BAD_RP0, NOT_MONOTONE, COL_RANGE, SELF_LOOP, NOT_ASCENDING, NOT_SYMMETRIC = range(7)


def csr_from_rows(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    return len(rows), rp, col


def code(rows=None, n=None, rp=None, col=None):
    if rows is not None:
        n, rp, col = csr_from_rows(rows)
    return oracle.check_csr(n, rp, col)


def test_valid_graphs():
    assert code([[1, 2], [0], [0]]) == OK
    assert code([[]]) == OK                      # one isolated vertex
    assert code([[], [], []]) == OK
    g = graphgen.rmat(10)
    assert oracle.check_csr(g.n, g.row_ptr, g.col) == OK


def test_row_ptr_not_starting_at_zero():
    n, rp, col = csr_from_rows([[1], [0]])
    rp2 = rp.copy()
    rp2[0] = 1
    assert code(n=n, rp=rp2, col=np.array([1, 1, 0], dtype=np.int32)) == BAD_RP0


def test_row_ptr_not_monotone():
    rp = np.array([0, 2, 1, 3], dtype=np.int32)
    col = np.array([1, 2, 0], dtype=np.int32)
    assert code(n=3, rp=rp, col=col) == NOT_MONOTONE


@pytest.mark.parametrize("bad", [-1, 3, 1000])
def test_column_out_of_range(bad):
    assert code([[1], [0, bad], []]) == COL_RANGE


def test_self_loop():
    assert code([[1], [0, 1]]) == SELF_LOOP
    assert code([[0]]) == SELF_LOOP


def test_unsorted_row():
    assert code([[2, 1], [0], [0]]) == NOT_ASCENDING


def test_duplicate_entry():
    assert code([[1, 1], [0]]) == NOT_ASCENDING


def test_missing_reverse_edge():
    assert code([[1, 2], [0], []]) == NOT_SYMMETRIC   # 0 -> 2 without 2 -> 0
    assert code([[1], []]) == NOT_SYMMETRIC


def test_grid_with_one_reverse_edge_removed():
    g = graphgen.grid(16)
    assert oracle.check_csr(g.n, g.row_ptr, g.col) == OK
    rows = [list(g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    u = 100
    v = rows[u][0]
    rows[v].remove(u)
    assert code(rows) == NOT_SYMMETRIC


def _valid_by_sets(n, rp, col):
    """Set-based definition: every row strictly ascending inside [0, n) minus
    the vertex itself, and the set of (u, v) pairs equal to its transpose."""
    if rp[0] != 0 or any(rp[v + 1] < rp[v] for v in range(n)):
        return False
    pairs = set()
    for v in range(n):
        row = [int(x) for x in col[rp[v]:rp[v + 1]]]
        if any(c < 0 or c >= n or c == v for c in row):
            return False
        if row != sorted(set(row)):
            return False
        pairs.update((v, c) for c in row)
    return pairs == {(b, a) for a, b in pairs}


def test_random_arrays_against_set_definition():
    rs = np.random.default_rng(3)
    seen = {True: 0, False: 0}
    for trial in range(3000):
        n = int(rs.integers(1, 7))
        A = rs.random((n, n)) < 0.4
        if trial % 2 == 0:
            A = A | A.T                   # symmetric half the time
        if trial % 5 != 0:
            np.fill_diagonal(A, False)    # loops in one trial of five
        rows = [list(np.nonzero(A[v])[0]) for v in range(n)]
        kind = trial % 7
        v = int(rs.integers(0, n))
        if kind == 1 and rows[v]:
            rows[v].append(rows[v][-1])   # duplicate
        elif kind == 2 and len(rows[v]) > 1:
            rows[v] = rows[v][::-1]       # unsorted
        elif kind == 3 and rows[v]:
            rows[v][-1] = n               # out of range
        nn, rp, col = csr_from_rows(rows)
        expect = _valid_by_sets(nn, rp, col)
        got = oracle.check_csr(nn, rp, col)
        assert (got == OK) == expect, (trial, rows, got)
        seen[expect] += 1
    assert seen[True] > 200 and seen[False] > 200
