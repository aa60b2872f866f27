"""Tuned schedules kept across processes (the autotuner's cache saved as JSON
keyed by a graph checksum): host logic, no GPU."""
import ctypes

import numpy as np
import pytest

import graphgen
import paper_2012_07990_amd as gg


def _all_schedules():
    out = []
    for algo in range(5):
        for preset in range(4):
            s = gg.Schedule()
            if gg._lib.gg_schedule_preset(algo, preset, ctypes.byref(s)) == gg.OK:
                out.append(s)
    s = gg.make_schedule(lb="strict", direction=gg.PULL, edge_blocking=True, blocking_size=777)
    s.threshold = 0.0123  # not exact in float32: must round-trip to the same float32
    out.append(s)
    return out


def test_schedule_dict_round_trip_is_exact():
    for s in _all_schedules():
        back = gg.schedule_from_dict(gg.schedule_to_dict(s))
        assert bytes(back) == bytes(s)


def test_checksum_sees_every_part_of_the_graph():
    g = graphgen.rmat(8, weights=True)
    base = gg.csr_checksum(g.n, g.row_ptr, g.col, g.w)
    assert base == gg.csr_checksum(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    col = g.col.copy()
    col[5] ^= 1
    assert gg.csr_checksum(g.n, g.row_ptr, col, g.w) != base
    w = g.w.copy()
    w[0] += 1
    assert gg.csr_checksum(g.n, g.row_ptr, g.col, w) != base
    assert gg.csr_checksum(g.n, g.row_ptr, g.col, None) != base
    assert gg.csr_checksum(g.n + 1, g.row_ptr, g.col, g.w) != base


def test_store_keeps_graphs_and_algorithms_apart(tmp_path):
    path = str(tmp_path / "tuned.json")
    a, b = _all_schedules()[0], _all_schedules()[-1]
    assert gg.load_tuned(path, "g1") == {}
    gg.save_tuned(path, "g1", gg.ALGO_BFS, a, 1.5)
    gg.save_tuned(path, "g1", gg.ALGO_PR, b, 12.5)
    gg.save_tuned(path, "g2", gg.ALGO_BFS, b, 2.0)
    got = gg.load_tuned(path, "g1")
    assert set(got) == {gg.ALGO_BFS, gg.ALGO_PR}
    assert bytes(got[gg.ALGO_BFS][0]) == bytes(a) and got[gg.ALGO_BFS][1] == 1.5
    assert bytes(got[gg.ALGO_PR][0]) == bytes(b)
    gg.save_tuned(path, "g1", gg.ALGO_BFS, b, 0.5)  # replaces, keeps the rest
    got = gg.load_tuned(path, "g1")
    assert bytes(got[gg.ALGO_BFS][0]) == bytes(b) and got[gg.ALGO_BFS][1] == 0.5
    assert set(gg.load_tuned(path, "g2")) == {gg.ALGO_BFS}


def test_tuned_cache_calls_reject_a_null_graph():
    s = gg.Schedule()
    assert gg._lib.gg_tuned_set(None, gg.ALGO_BFS, ctypes.byref(s), 1.0) == gg.ERR_INVALID_ARG
    assert gg._lib.gg_tuned_get(None, gg.ALGO_BFS, ctypes.byref(s), None) == gg.ERR_INVALID_ARG
