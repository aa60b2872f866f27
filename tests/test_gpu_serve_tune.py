"""GPU: the serving loop (every result identical to the same query run alone,
batching happens, admission refuses queries that can never fit) and the
autotuner (returns a valid schedule whose result matches the oracle)."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2012_07990_amd as gg
from gpu_util import assert_int_equal, dev_graph, host_graph, oracle_bc, oracle_bfs, oracle_sssp

pytestmark = pytest.mark.gpu


def _alone(G, algo, src):
    if algo == gg.ALGO_BFS:
        return G.bfs(src, gg.schedule_preset(gg.ALGO_BFS, gg.PRESET_POWERLAW)).cpu().numpy().view(np.uint8)
    if algo == gg.ALGO_SSSP:
        s = gg.schedule_preset(gg.ALGO_SSSP, gg.PRESET_POWERLAW)
        s.s1.delta = 64
        return G.sssp(src, s).cpu().numpy().view(np.uint8)
    sig, dl = G.bc(src, gg.schedule_preset(gg.ALGO_BC, gg.PRESET_POWERLAW))
    return np.concatenate([sig.cpu().numpy().view(np.uint8), dl.cpu().numpy().view(np.uint8)])


def test_serving_mix_identical_to_alone():
    names = ["rmat12", "rmat14", "grid64"]
    Gs = [dev_graph(n) for n in names]
    srv = gg.Server(budget_bytes=1 << 30, nstreams=4)
    gids = [srv.add_graph(G) for G in Gs]
    rng = np.random.default_rng(3)
    queries = []
    for i in range(300):
        gi = int(rng.integers(0, 3))
        algo = [gg.ALGO_BFS, gg.ALGO_BFS, gg.ALGO_SSSP, gg.ALGO_BC][int(rng.integers(0, 4))]
        if algo == gg.ALGO_BC and names[gi] == "grid64":
            algo = gg.ALGO_BFS  # path counts on grids overflow 64 bits
        src = int(rng.integers(0, Gs[gi].n))
        queries.append((gi, algo, src, srv.submit(gids[gi], algo, src)))
    batched = 0
    for gi, algo, src, t in queries:
        n = Gs[gi].n
        out = np.empty(12 * n if algo == gg.ALGO_BC else 4 * n, dtype=np.uint8)
        r = srv.wait(t, 60.0, out=out)
        assert r is not None and r["status"] == gg.OK
        batched += r["batch_size"] > 1
        assert np.array_equal(out, _alone(Gs[gi], algo, src)), (names[gi], algo, src)
        if algo == gg.ALGO_BFS:
            assert_int_equal(out.view(np.int32), oracle_bfs(names[gi], src))
    st = srv.stats()
    assert st["completed"] == 300 and st["collected"] == 300 and st["bytes_in_use"] == 0
    assert st["max_batch"] > 1 and batched > 0
    srv.close()


def test_serving_admission_and_errors():
    G = dev_graph("rmat12")
    srv = gg.Server(budget_bytes=1 << 10, nstreams=1)
    gid = srv.add_graph(G)
    with pytest.raises(gg.GGError) as e:
        srv.submit(gid, gg.ALGO_BFS, 0)
    assert e.value.status == gg.ERR_ADMISSION
    with pytest.raises(gg.GGError) as e:
        srv.submit(gid, gg.ALGO_BFS, G.n)
    assert e.value.status == gg.ERR_INVALID_ARG
    with pytest.raises(gg.GGError) as e:
        srv.poll(12345)
    assert e.value.status == gg.ERR_NOT_FOUND
    with pytest.raises(gg.GGError) as e:
        srv.set_schedule(gid, gg.ALGO_BFS, gg.make_schedule(lb="twc", fusion=True))
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    srv.close()


def test_serving_fused_schedule_runs_exclusively():
    names = ["grid64", "rmat12"]
    Gs = [dev_graph(n) for n in names]
    srv = gg.Server(budget_bytes=1 << 30, nstreams=3)
    gids = [srv.add_graph(G) for G in Gs]
    srv.set_schedule(gids[0], gg.ALGO_SSSP, gg.make_schedule(lb="cm", delta=64, fusion=True))
    qs = []
    for i in range(60):
        gi = i % 2
        algo = gg.ALGO_SSSP if i % 3 else gg.ALGO_BFS
        src = (i * 37) % Gs[gi].n
        qs.append((gi, algo, src, srv.submit(gids[gi], algo, src)))
    for gi, algo, src, t in qs:
        out = np.empty(Gs[gi].n, dtype=np.int32)
        r = srv.wait(t, 60.0, out=out)
        assert r["status"] == gg.OK
        exp = oracle_sssp(names[gi], src) if algo == gg.ALGO_SSSP else oracle_bfs(names[gi], src)
        assert_int_equal(out, exp)
    srv.close()


def test_serving_batches_sssp_and_reports_overflow_per_query():
    G = dev_graph("grid64")
    srv = gg.Server(budget_bytes=1 << 30, nstreams=2)
    gid = srv.add_graph(G)
    ts = [(s, srv.submit(gid, gg.ALGO_SSSP, s)) for s in range(0, 4096, 41)]
    batched = 0
    for s, t in ts:
        out = np.empty(G.n, dtype=np.int32)
        r = srv.wait(t, 60.0, out=out)
        assert r["status"] == gg.OK
        batched += r["batch_size"] > 1
        assert_int_equal(out, oracle_sssp("grid64", s))
    assert batched > 0
    srv.close()
    # path of 4 with huge weights: from vertex 0 the far end is beyond INT32_MAX-1,
    # from vertex 1 every distance fits
    g = graphgen.path(4)
    H = gg.Graph.from_csr(g.n, g.row_ptr, g.col, np.full(g.m, 999_999_999, dtype=np.uint32))
    srv = gg.Server(budget_bytes=1 << 30, nstreams=1)
    gid = srv.add_graph(H)
    ts = [(s, srv.submit(gid, gg.ALGO_SSSP, s)) for s in [0, 1, 3, 2, 0, 1]]
    for s, t in ts:
        out = np.empty(4, dtype=np.int32)
        if s in (0, 3):
            with pytest.raises(gg.GGError) as e:
                srv.wait(t, 60.0, out=out)
            assert e.value.status == gg.ERR_OVERFLOW
            continue
        r = srv.wait(t, 60.0, out=out)
        assert r["status"] == gg.OK
        if s == 1:
            assert list(out) == [999_999_999, 0, 999_999_999, 1_999_999_998]
    srv.close()


def test_serving_small_budget_still_completes():
    G = dev_graph("rmat12")
    one = G.workspace_bytes(gg.ALGO_BFS, 1) + 4 * G.n
    srv = gg.Server(budget_bytes=3 * one, nstreams=2)
    gid = srv.add_graph(G)
    ts = [srv.submit(gid, gg.ALGO_BFS, s) for s in range(40)]
    for s, t in enumerate(ts):
        out = torch.empty(G.n, dtype=torch.int32, device="cuda")
        r = srv.wait(t, 60.0, out=out)
        assert r["status"] == gg.OK
        assert_int_equal(out.cpu().numpy(), oracle_bfs("rmat12", s))
    assert srv.stats()["bytes_peak"] <= 3 * one
    srv.close()


@pytest.mark.parametrize("algo", [gg.ALGO_BFS, gg.ALGO_SSSP, gg.ALGO_CC, gg.ALGO_PR, gg.ALGO_BC])
def test_autotune_returns_valid_schedule(algo):
    name = "rmat12"
    G = dev_graph(name)
    src = graphgen.max_degree_vertex(host_graph(name))
    s, ms = G.autotune(algo, budget_s=3.0, probes=[src, 0])
    assert ms > 0
    G.validate(algo, s)
    s2, ms2 = G.autotune(algo, budget_s=0.0)  # cached
    assert bytes(s2) == bytes(s) and ms2 == ms
    if algo == gg.ALGO_BFS:
        assert_int_equal(G.bfs(src, s).cpu().numpy(), oracle_bfs(name, src))
    elif algo == gg.ALGO_SSSP:
        assert_int_equal(G.sssp(src, s).cpu().numpy(), oracle_sssp(name, src))
    elif algo == gg.ALGO_BC:
        sig, _ = G.bc(src, s)
        assert_int_equal(sig.cpu().numpy().view(np.uint64), oracle_bc(name, src)[0])


def test_tuned_schedule_survives_a_new_graph_object(tmp_path):
    """The autotuner's winner, saved as JSON under the graph's checksum, seeds
    a fresh graph of the same CSR: gg_autotune with no budget returns it
    unchanged, and it runs to the oracle's result."""
    h = host_graph("rmat12")
    G = dev_graph("rmat12")
    src = graphgen.max_degree_vertex(h)
    s, ms = G.autotune(gg.ALGO_BFS, budget_s=1.0, probes=[src])
    key = gg.csr_checksum(h.n, h.row_ptr, h.col, h.w)
    path = str(tmp_path / "tuned.json")
    assert G.save_tuned(path, key) >= 1
    G2 = gg.Graph.from_graphgen(h)
    assert G2.tuned(gg.ALGO_BFS) is None
    assert G2.load_tuned(path, key) >= 1
    s2, ms2 = G2.autotune(gg.ALGO_BFS, budget_s=0.0)
    assert bytes(s2) == bytes(s) and ms2 == pytest.approx(ms)
    assert_int_equal(G2.bfs(src, s2).cpu().numpy(), oracle_bfs("rmat12", src))
    with pytest.raises(gg.GGError) as e:
        G2.set_tuned(gg.ALGO_PR, gg.make_schedule(lb="vp", direction=gg.PUSH))
    assert e.value.status == gg.ERR_UNSUPPORTED_SCHEDULE
    G2.close()
