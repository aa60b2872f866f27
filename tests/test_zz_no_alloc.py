"""gg_bfs_noalloc (workspace carved from a fixed device array, no allocation)
against gg_bfs (pooled workspace) through the C ABI: the same depths, bit for
bit, on two calls in a row with the second on a smaller graph (the array keeps
the first call's contents), under every schedule family it accepts, plus its
refusals. The depths are also checked against the oracle."""
import ctypes

import pytest

import graphgen
import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal, dev_graph, oracle_bfs, source

pytestmark = pytest.mark.gpu


def _hybrid(lb):
    s = gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)
    s.s1.load_balance = gg.LB_NAMES[lb]
    s.threshold = 0.01
    return s


SCHEDULES = {
    "push-vp": lambda: gg.make_schedule(lb="vp"),
    "push-strict": lambda: gg.make_schedule(lb="strict"),
    "push-twc-boolmap": lambda: gg.make_schedule(lb="twc", creation=gg.CREATE_UNFUSED_BOOLMAP),
    "push-etwc-bitmapdedup": lambda: gg.make_schedule(lb="etwc", dedup_type=gg.DEDUP_BITMAP),
    "push-cm-boolmapdedup": lambda: gg.make_schedule(lb="cm", dedup_type=gg.DEDUP_BOOLMAP),
    "hybrid-strict": lambda: _hybrid("strict"),
    "pull": lambda: gg.make_schedule(direction=gg.PULL),
    "fused-cm": lambda: gg.make_schedule(lb="cm", fusion=True),
    "fused-hybrid": lambda: gg.make_schedule(lb="vp", fusion=True, threshold=0.01,
                                             hybrid={"direction": gg.PULL, "pull_rep": gg.REP_BITMAP}),
}


def _noalloc(name, sched, src):
    import torch
    G = dev_graph(name)
    out = torch.full((G.n,), 12345, dtype=torch.int32, device="cuda")
    gg.gg_bfs_noalloc(G, src, sched, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("key", sorted(SCHEDULES))
def test_noalloc_matches_bfs_twice_second_smaller(key):
    sched = SCHEDULES[key]()
    for name in ["rmat16", "rmat12"]:  # the second call runs on a smaller graph
        src = source(name)
        ref = dev_graph(name).bfs(src, sched).cpu().numpy()
        got = _noalloc(name, sched, src)
        assert_int_equal(got, ref, "noalloc vs gg_bfs %s %s" % (key, name))
        assert_int_equal(got, oracle_bfs(name, src), "noalloc vs oracle %s %s" % (key, name))


def test_noalloc_high_diameter_and_degenerate():
    for name in ["grid64", "path100k", "isolated7", "single", "star5000"]:
        src = source(name)
        s = gg.make_schedule(lb="cm", fusion=True) if name in ("grid64", "path100k") else gg.make_schedule()
        assert_int_equal(_noalloc(name, s, src), dev_graph(name).bfs(src, s).cpu().numpy(), name)


def test_noalloc_refusals():
    import torch
    G = dev_graph("rmat12")
    out = torch.empty(G.n, dtype=torch.int32, device="cuda")
    st = gg._lib.gg_bfs_noalloc(G.handle, 0, gg._sched_ptr(gg.make_schedule(lb="edge_only")),
                                ctypes.c_void_p(out.data_ptr()), None)
    assert st == gg.ERR_UNSUPPORTED_SCHEDULE
    st = gg._lib.gg_bfs_noalloc(G.handle, G.n, None, ctypes.c_void_p(out.data_ptr()), None)
    assert st == gg.ERR_INVALID_ARG
    big = gg.Graph.from_graphgen(graphgen.isolated((1 << 20) + 1))  # one vertex past the limit
    out_big = torch.empty(big.n, dtype=torch.int32, device="cuda")
    st = gg._lib.gg_bfs_noalloc(big.handle, 0, None, ctypes.c_void_p(out_big.data_ptr()), None)
    assert st == gg.ERR_INVALID_ARG and "vertices" in gg._lib.gg_last_error().decode()
    big.close()
    # still usable after the refusals
    src = source("rmat12")
    assert_int_equal(_noalloc("rmat12", gg.make_schedule(lb="strict"), src), oracle_bfs("rmat12", src), "after")
