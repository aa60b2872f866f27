"""C-ABI surface checks that need no GPU: the library loads, exports every
function the header declares, and rejects bad arguments before touching HIP."""
import ctypes

import pytest

import paper_2012_07990_amd as gg


def test_exports_every_header_function():
    names = gg.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(gg._lib, n), "libgg.so does not export %s" % n


def test_status_strings_and_version():
    assert gg.status_string(gg.OK) == "ok"
    assert gg.status_string(gg.ERR_UNSUPPORTED_SCHEDULE) == "unsupported schedule"
    assert "gfx950" in gg.version()


def test_schedule_defaults_follow_the_table():
    s = gg.schedule_default()
    assert s.hybrid == 0
    s1 = s.s1
    assert s1.load_balance == gg.LB_VERTEX_BASED and s1.direction == gg.PUSH
    assert s1.pull_rep == gg.REP_BOOLMAP and s1.frontier_creation == gg.CREATE_FUSED
    assert s1.dedup_enable == 1 and s1.dedup_type == gg.DEDUP_MONOTONIC_COUNTERS
    assert s1.kernel_fusion == 0


def test_bfs_hybrid_preset():
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_BFS_HYBRID)
    assert s.hybrid == 1
    assert s.s1.direction == gg.PUSH and s.s1.load_balance == gg.LB_VERTEX_BASED
    assert s.s2.direction == gg.PULL and s.s2.pull_rep == gg.REP_BITMAP
    assert s.s2.dedup_enable == 0 and s.s2.frontier_creation == gg.CREATE_UNFUSED_BITMAP


def test_create_rejects_bad_sizes_without_gpu():
    h = ctypes.c_void_p()
    rp = (ctypes.c_int32 * 2)(0, 0)
    st = gg._lib.gg_graph_create_csr(0, 0, rp, None, None, 0, None, ctypes.byref(h))
    assert st == gg.ERR_INVALID_ARG and "n must be" in gg._lib.gg_last_error().decode()
    st = gg._lib.gg_graph_create_csr(1, -1, rp, None, None, 0, None, ctypes.byref(h))
    assert st == gg.ERR_INVALID_ARG
    st = gg._lib.gg_graph_create_csr(1, 0, None, None, None, 0, None, ctypes.byref(h))
    assert st == gg.ERR_INVALID_ARG
    st = gg._lib.gg_graph_create_csr(1, 0, rp, None, None, 0, None, None)
    assert st == gg.ERR_INVALID_ARG


def test_null_graph_rejected():
    assert gg._lib.gg_bfs(None, 0, None, None, None, None) == gg.ERR_INVALID_ARG
    assert gg._lib.gg_graph_destroy(None) == gg.OK


def test_preset_rejects_unknown():
    s = gg.Schedule()
    assert gg._lib.gg_schedule_preset(0, 99, ctypes.byref(s)) == gg.ERR_INVALID_ARG


def test_python_constants_match_the_header():
    """Every GG_* #define and enumerator in include/gg.h has the same value
    under its unprefixed name in the Python binding."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "gg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", " ", hdr, flags=re.S)
    found = {}
    for name, val in re.findall(r"#define\s+GG_(\w+)\s+(\d+)u?\b", hdr):
        found[name] = int(val)
    for body in re.findall(r"typedef\s+enum\s*\{(.*?)\}", hdr, flags=re.S):
        for name, val in re.findall(r"GG_(\w+)\s*=\s*(\d+)", body):
            found[name] = int(val)
    assert "PR_NO_LDS_CACHE" in found and "LB_EDGE_ONLY" in found
    missing = [n for n in found if not hasattr(gg, n)]
    assert not missing, "binding lacks %s" % missing
    wrong = {n: (found[n], getattr(gg, n)) for n in found if getattr(gg, n) != found[n]}
    assert not wrong, wrong
