"""The algorithm-language compiler on the CPU: parsing, schedule lowering,
the analyses that pick atomics and rewrite frontier handling, refusals of
programs outside the supported subset, and that every example variant was
built into a module exporting gen_main. No GPU needed."""
import ctypes
import os
import re

import pytest

from paper_2012_07990_amd import compiler
from paper_2012_07990_amd.compiler import CompileError, compile_source, parse, variant_source


def gen(name):
    return compile_source(variant_source(name), compiler.VARIANTS[name][1])


def functor(code, prefix):
    """Body of the first generated struct whose name starts with prefix."""
    m = re.search(r"struct (%s\w*) \{(.*?)\n\};" % prefix, code, re.S)
    assert m, prefix
    return m.group(2)


def test_parse_examples():
    for f in ("bfs.gt", "sssp.gt", "cc.gt", "pagerank.gt"):
        p = parse(open(os.path.join(compiler.EXAMPLES, f)).read())
        assert "main" in p.funcs and p.edges is not None and p.vertices == "vertices"
    p = parse(open(os.path.join(compiler.EXAMPLES, "sssp.gt")).read())
    assert p.edges["weighted"] and p.vectors["dist"]["type"] == "int"
    p = parse(open(os.path.join(compiler.EXAMPLES, "pagerank.gt")).read())
    assert set(p.vectors) == {"old_rank", "new_rank", "contrib", "out_degree"}
    assert set(p.scalars) == {"damp", "beta_score", "init_rank"}


def test_atomic_insertion():
    # BFS push: the filter tests parent[v] == -1 and the function writes parent[dst] -> one CAS
    code, notes = gen("bfs_push_twce")
    push = functor(code, "E_updateEdge_push")
    assert "atomic_cas_i32(&vec_parent[v], (-1)" in push
    pull = functor(code, "E_updateEdge_pull")
    assert "atomic" not in pull and "done(int v) const { return !((vec_parent[v] == (-1))); }" in pull
    assert any("compare-and-swap" in n for n in notes)
    # SSSP and CC: min= -> atomic minimum when pushing, a plain compare-and-write when pulling
    for name, vec in (("sssp_push_strict", "dist"), ("cc_push_etwc", "IDs")):
        code, _ = gen(name)
        assert "atomic_min_i32(&vec_%s[v]" % vec in functor(code, "E_updateEdge_push")
        assert "atomic" not in functor(code, "E_updateEdge_pull")
    # PageRank: += -> atomic add when pushing, a plain add (one lane per destination) when pulling
    code, _ = gen("pagerank_pull")
    assert "atomic_add_f64(&vec_new_rank[v]" in functor(code, "E_updateEdge_push")
    pull = functor(code, "E_updateEdge_pull")
    assert "vec_new_rank[v] += " in pull and "atomic" not in pull


def test_frontier_reuse_and_loops():
    code, notes = gen("bfs_push_twce")
    assert any("double-buffer swap" in n for n in notes)
    assert code.count("FrontierState fs(") == 1          # one frontier, allocated once
    assert "while (fs.count > 0)" in code
    code, _ = gen("pagerank_pull")
    assert "for (int64_t h_i = 0; h_i < 20; h_i++)" in code
    assert "gen::out_degrees<int32_t>" in code and "FrontierState" not in code
    # deduplication disabled -> the queue can hold every emitted (vertex, edge) pair
    code, _ = gen("sssp_push_vp_nodedup")
    assert "FrontierState fs(c, *ws, g.n, (long long)g.n + g.m);" in code
    code, _ = gen("sssp_push_strict")
    assert "FrontierState fs(c, *ws, g.n, (long long)g.n);" in code


def _sched(code):
    m = re.search(r"const gg_schedule sch_s1 = gg_schedule\{(.*)\};", code)
    return m.group(1)


def test_schedule_lowering():
    s = _sched(gen("bfs_push_twce")[0])
    assert s.startswith("0, ") and "{GG_LB_ETWC, 0, 1048576, GG_PUSH, GG_REP_BOOLMAP, GG_CREATE_FUSED, 1, " \
                                  "GG_DEDUP_MONOTONIC_COUNTERS" in s
    s = _sched(gen("bfs_push_strict_boolmap")[0])
    assert "{GG_LB_STRICT, 0, 1048576, GG_PUSH, GG_REP_BOOLMAP, GG_CREATE_UNFUSED_BOOLMAP," in s
    s = _sched(gen("bfs_pull_bitmap")[0])
    assert "GG_PULL, GG_REP_BITMAP, GG_CREATE_UNFUSED_BITMAP" in s
    s = _sched(gen("bfs_hybrid")[0])
    assert s.startswith("1, 0.05f, {GG_LB_ETWC,") and s.count("GG_PULL, GG_REP_BITMAP") == 1
    s = _sched(gen("sssp_push_vp_nodedup")[0])
    assert "{GG_LB_VERTEX_BASED, 0, 1048576, GG_PUSH, GG_REP_BOOLMAP, GG_CREATE_FUSED, 0," in s
    s = _sched(gen("cc_push_edge_only")[0])
    assert "GG_LB_EDGE_ONLY" in s
    code, _ = gen("cc_push_edge_only")
    assert "ensure_coo(c, G);" in code
    code, _ = gen("sssp_pull")
    assert "require(G.symmetric, GG_ERR_UNSUPPORTED_SCHEDULE" in code and "ensure_transpose(c, G);" in code
    code, _ = gen("bfs_pull_bitmap")
    assert "ensure_transpose(c, G);" in code and "require(G.symmetric" not in code


def test_kernel_fusion_lowering():
    code, notes = gen("bfs_fused_hybrid_strict")
    assert "gen::fused_loop<GG_LB_STRICT, kDedupMonotonic, 2>(c, G, g, *ws, fs, 0.05f, " \
           "E_updateEdge_push_toFilter_parent" in code
    assert "while (fs.count > 0)" not in code          # the loop runs on the device
    assert any("one persistent launch" in n for n in notes)
    code, _ = gen("bfs_fused_wm_boolpull")
    assert "gen::fused_loop<GG_LB_WM, kDedupMonotonic, 1>(c, G, g, *ws, fs, 0.02f," in code
    # fusion requested on the operator's own schedule, deduplication off
    code, _ = gen("sssp_fused_vp_nodedup")
    assert "gen::fused_loop<GG_LB_VERTEX_BASED, kDedupNone, 0>(c, G, g, *ws, fs, 0.0f," in code
    assert "FrontierState fs(c, *ws, g.n, (long long)g.n + g.m);" in code
    code, _ = gen("cc_fused_cm")
    assert "gen::fused_loop<GG_LB_CM, kDedupMonotonic, 0>" in code


FUSE = """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    %s
    program->applyGPUSchedule("s1", s1);"""


@pytest.mark.parametrize("cfg,match", [
    ("s1.configLoadBalance(TWC);", "VERTEX_BASED, WM, CM, STRICT or ETWC"),
    ("s1.configLoadBalance(EDGE_ONLY);", "VERTEX_BASED, WM, CM, STRICT or ETWC"),
    ("s1.configDirection(PULL);", "PUSH steps"),
    ("s1.configFrontierCreation(UNFUSED_BITMAP);", "PUSH steps"),
    ("s1.configDeduplication(ENABLED, BITMAP);", "monotonic counters"),
])
def test_kernel_fusion_refusals(cfg, match):
    src = variant_source("bfs_push_twce")
    src = src[:src.index("schedule:")] + "schedule:" + FUSE % cfg + "\n"
    with pytest.raises(CompileError, match=match):
        compile_source(src, ["parent"])


def test_fused_loop_statements():
    # a vector element written from the host cannot run inside the fused loop
    src = variant_source("bfs_fused_hybrid_strict").replace(
        "        delete frontier;\n        frontier = output;\n    end",
        "        delete frontier;\n        frontier = output;\n        parent[0] = 0;\n    end")
    with pytest.raises(CompileError, match="cannot run inside a fused loop"):
        compile_source(src, ["parent"])
    # nor a scalar statement that reads vertex data
    src = variant_source("bfs_rounds_fused").replace("rounds = rounds + 1;", "rounds = parent[0];")
    with pytest.raises(CompileError, match="local variables and literals"):
        compile_source(src, ["parent"])


def test_fused_loop_hoisting():
    code, notes = gen("bfs_rounds_fused")
    # one generated persistent kernel with the loop, main's locals hoisted in and out
    assert "__global__ __launch_bounds__(kBlock) void k_fused_0(gen::GenFusedArgs a," in code
    assert "int64_t h_rounds = hoist[0];" in code and "hoist[1] = h_work;" in code
    assert "gen::fused_vertices(a.g.n, vf0, s.t);" in code
    assert "gen::fused_step<GG_LB_STRICT, kDedupMonotonic, 2>(a, fp, fl, s, cnt)" in code
    k = code.index("void k_fused_0")
    body = code[k:code.index("\n}\n", k)]
    # statement order of the loop body: counter, vertex apply + barrier, operator, recurrence, tail
    order = [body.index(x) for x in ("h_rounds = (h_rounds + 1);", "gen::fused_vertices", "grid_sync(s.bar)",
                                     "gen::fused_step", "h_work = ((h_work + (2 * h_rounds)) - 1);",
                                     "gen::fused_round_tail")]
    assert order == sorted(order)
    assert any("hoisted to device memory: rounds, work" in n for n in notes)
    # the unfused form runs the same statements on the host around the operator
    code, _ = gen("bfs_rounds")
    assert "h_rounds += 0" not in code and "h_rounds = (h_rounds + 1);" in code
    assert "while (fs.count > 0)" in code and "k_fused_" not in code


def test_edge_blocking():
    # every edge processed (edges.apply): the EdgeBlocked COO, one launch per segment
    code, notes = gen("pagerank_push_blocked")
    assert "gen::all_edges_blocked(c, G, 1000, E_updateEdge_push{" in code
    assert any("destination segments of 1000 vertices" in n for n in notes)
    # a frontier operator processes a frontier's edges only: refused
    src = variant_source("cc_push_edge_only").replace("configLoadBalance(EDGE_ONLY)",
                                                      "configLoadBalance(EDGE_ONLY, BLOCKED, 65536)")
    with pytest.raises(CompileError, match="every edge is processed"):
        compile_source(src, ["IDs"])


PQ = open(os.path.join(compiler.EXAMPLES, "sssp_pq.gt")).read()


def test_priority_queue_lowering():
    code, notes = gen("sssp_pq_strict_d64")
    f = functor(code, "P_relax_pq")
    # the candidate is summed in 64 bits; the update is the queue's atomic-minimum bucket test
    assert "const int64_t l_candidate = (int64_t)(((int64_t)vec_dist[u] + (int64_t)w[e]));" in f
    assert "gen::pq_update_min(pq, v, (long long)(l_candidate), tf_0)" in f
    assert "wave_append(pq.farq, pq.farc, pq.far_cap, pq.flags + 1, tf_0, v);" in f
    assert "gen::pq_start(c, *ws, fs, pq_pq, 64);" in code
    assert "while (gen::pq_next(c, *ws, fs, pq_pq, iter))" in code
    assert any("buckets of width 64 (configDelta)" in n for n in notes)
    assert "gen::pq_start(c, *ws, fs, pq_pq, 1);" in gen("sssp_pq_etwc_d1")[0]
    assert "gen::pq_start(c, *ws, fs, pq_pq, 4096);" in gen("sssp_pq_cm_d4096_boolmap")[0]


@pytest.mark.parametrize("edit,match", [
    (("s1.configDelta(64);", "s1.configDelta(64);\n    s1.configDirection(PULL);"), "unfused PUSH"),
    (("s1.configDelta(64);", "s1.configDelta(64);\n    s1.configKernelFusion(ENABLED);"), "unfused PUSH"),
    (("pq = new priority_queue{Vertex}(int)(dist, start_vertex);\n", ""), "before it is created"),
    (("        delete frontier;\n    end", "    end"), "loop of pq holds"),
    (("pq.updatePriorityMin(dst, candidate);", "dist[dst] min= candidate;"), "updatePriorityMin"),
])
def test_priority_queue_refusals(edit, match):
    with pytest.raises(CompileError, match=match):
        compile_source(PQ.replace(*edit), ["dist"])


def test_host_writes_are_checked():
    code, _ = gen("bfs_push_twce")
    assert "gen::set_one<int32_t>(c, vec_parent.p, g.n, (int64_t)(h_start_vertex)" in code
    assert "gen::add_vertex(c, fs, g.n, (int64_t)(h_start_vertex));" in code
    assert 'require(outs[0] != nullptr' in code


def test_generation_is_deterministic():
    for name in compiler.VARIANTS:
        assert gen(name)[0] == gen(name)[0]


BFS = open(os.path.join(compiler.EXAMPLES, "bfs.gt")).read()


def _with_main(body):
    head = BFS[:BFS.index("func main()")]
    return head + "func main()\n" + body + "\nend\n"


@pytest.mark.parametrize("src,match", [
    ("element Vertex end\nfunc main()\nend\n", "no edgeset"),
    (BFS.replace("func main()", "func notmain()"), "no main"),
    (BFS.replace("const parent : vector{Vertex}(int) = -1;",
                 "const parent : vector{Vertex}(int) = -1;\nconst pq : priority_queue{Vertex}(int) = 0;"),
     "created in main"),
    (_with_main("""
    var frontier : vertexset{Vertex} = new vertexset{Vertex}(0);
    frontier.addVertex(0);
    while (frontier.getVertexSetSize() != 0)
        #s1# var output : vertexset{Vertex} = edges.from(frontier).to(toFilter).applyModified(updateEdge, parent, true);
        frontier = output;
    end"""), "delete frontier"),
    (BFS.replace("s1.configLoadBalance(TWCE);", "s1.configLoadBalance(NOT_A_STRATEGY);"), "NOT_A_STRATEGY"),
    (BFS.replace("func updateEdge(src : Vertex, dst : Vertex)", "func updateEdge(src : Vertex, dst : Vertex, w : int)"),
     "unweighted"),
    (BFS.replace("parent[start_vertex] = start_vertex;", "parent[start_vertex] = start_vertex; @"),
     "unexpected character"),
])
def test_refusals(src, match):
    with pytest.raises(CompileError, match=match):
        compile_source(src, ["parent"])


def test_output_must_be_a_vector():
    with pytest.raises(CompileError, match="not a vector"):
        compile_source(BFS, ["depth"])


def test_examples_built():
    """build() compiled every variant; each module exports gen_main."""
    for name in compiler.VARIANTS:
        so = os.path.join(compiler.GEN_DIR, name + ".so")
        assert os.path.exists(so), "%s missing: run __graft_entry__.build()" % so
        lib = ctypes.CDLL(so)
        assert hasattr(lib, "gen_main")
