"""Compiler for programs in the algorithm and scheduling languages (the
subset of the Algorithm Language and Scheduling Language sections this
library runs): parse, lower the schedules and analyse the functions
(atomic insertion, enqueue rewriting, frontier reuse), emit HIP C++ against
the library's operator templates (csrc/gen_rt.hpp), compile it for gfx950
with hipcc into a module linked with libgg.so, and run its main through the
module's C entry point.

    from paper_2012_07990_amd import compiler
    mod = compiler.build_program(open("bfs.gt").read(), "bfs", outputs=["parent"])
    parent = mod.run(graph, args=[source])["parent"]

Compilation happens on the host (hipcc cross-compiles without a GPU);
running needs the device.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from typing import Dict, List, Optional, Sequence

from .codegen import generate
from .lang import CompileError, parse

__all__ = ["CompileError", "parse", "compile_source", "build_program", "load", "Module", "EXAMPLES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_PKG = os.path.dirname(_HERE)
_CSRC = os.path.join(_PKG, "csrc")
GEN_DIR = os.path.join(_PKG, "_gen")
EXAMPLES = os.path.join(_HERE, "examples")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

_FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-variable",
          "-Wno-unused-function", "-Wno-unused-but-set-variable"]


def compile_source(src: str, outputs: Sequence[str]):
    """(HIP C++ text, analysis notes) of a program; raises CompileError."""
    prog = parse(src)
    return generate(prog, list(outputs))


def _hash(text: str) -> str:
    """Key of a built module: the generated source and the headers it
    includes (which fix the layout of everything it shares with libgg.so)."""
    h = hashlib.sha256(text.encode())
    for f in sorted(os.listdir(_CSRC)):
        if f.endswith(".hpp") or f.endswith(".h"):
            with open(os.path.join(_CSRC, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(_PKG, "..", "include", "gg.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def build_program(src: str, name: str, outputs: Sequence[str], out_dir: Optional[str] = None,
                  force: bool = False) -> "Module":
    """Compile a program into <out_dir>/<name>.so (reused when the generated
    source is unchanged) and load it."""
    path = build_only(src, name, outputs, out_dir, force)
    return load(path, outputs)


def build_only(src: str, name: str, outputs: Sequence[str], out_dir: Optional[str] = None,
               force: bool = False) -> str:
    code, notes = compile_source(src, outputs)
    out_dir = out_dir or GEN_DIR
    os.makedirs(out_dir, exist_ok=True)
    cpp = os.path.join(out_dir, name + ".hip")
    so = os.path.join(out_dir, name + ".so")
    stamp = os.path.join(out_dir, name + ".sha")
    h = _hash(code)
    if not force and os.path.exists(so) and os.path.exists(stamp) and open(stamp).read().strip() == h:
        return so
    with open(cpp, "w") as fh:
        fh.write(code)
    with open(os.path.join(out_dir, name + ".notes"), "w") as fh:
        fh.write("\n".join(notes) + "\n")
    tmp = so + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-x", "hip"] + _FLAGS + ["-shared", "-I", _CSRC, cpp, "-o", tmp, "-L", _PKG, "-lgg",
                                           "-Wl,-rpath," + _PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise CompileError("hipcc failed for %s:\n%s" % (name, r.stderr[-8000:]))
    os.replace(tmp, so)
    with open(stamp, "w") as fh:
        fh.write(h + "\n")
    return so


class Module:
    """A compiled program: run(graph, args) executes its main on the graph
    and returns its output vectors (torch tensors on the device)."""

    def __init__(self, path: str, outputs: Sequence[str], types: Dict[str, str]):
        import paper_2012_07990_amd  # noqa: F401  (libgg.so first: the module links against it)
        self.path = path
        self.outputs = list(outputs)
        self.types = types
        self.lib = ctypes.CDLL(path)
        self.lib.gen_main.restype = ctypes.c_int
        self.lib.gen_main.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p]

    def run(self, graph, args: Sequence[int] = (), stream=None):
        import numpy as np
        import torch
        import paper_2012_07990_amd as gg
        tt = {"int": torch.int32, "bool": torch.int32, "float": torch.float32, "double": torch.float64}
        outs = {o: torch.empty(graph.n, dtype=tt[self.types[o]], device="cuda") for o in self.outputs}
        a = np.ascontiguousarray(np.asarray(list(args), dtype=np.int64))
        ptrs = (ctypes.c_void_p * max(len(self.outputs), 1))(*[ctypes.c_void_p(outs[o].data_ptr())
                                                              for o in self.outputs])
        st = self.lib.gen_main(graph.handle, ctypes.c_void_p(a.ctypes.data) if a.size else None, int(a.size),
                               ptrs, gg._stream(stream))
        if st != gg.OK:
            raise gg.GGError(st, "gen_main(%s)" % os.path.basename(self.path))
        return outs


def load(path: str, outputs: Sequence[str], src: Optional[str] = None) -> Module:
    if src is None:
        base = os.path.splitext(path)[0]
        hip = base + ".hip"
        types = {}
        if os.path.exists(hip):
            txt = open(hip).read()
            for o in outputs:
                for ct, ty in (("int32_t", "int"), ("double", "double"), ("float", "float")):
                    if "DevBuf<%s> vec_%s;" % (ct, o) in txt:
                        types[o] = ty
        return Module(path, outputs, types)
    prog = parse(src)
    return Module(path, outputs, {o: prog.vectors[o]["type"] for o in outputs})


# the example programs and the schedule variants the tests run (name -> (file, outputs, schedule section))
VARIANTS = {
    "bfs_push_twce": ("bfs.gt", ["parent"], None),
    "bfs_push_strict_boolmap": ("bfs.gt", ["parent"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(STRICT);
    s1.configFrontierCreation(UNFUSED_BOOLMAP);
    program->applyGPUSchedule("s1", s1);"""),
    "bfs_pull_bitmap": ("bfs.gt", ["parent"], """
    SimpleGPUSchedule s1;
    s1.configDirection(PULL, BITMAP);
    s1.configFrontierCreation(UNFUSED_BITMAP);
    program->applyGPUSchedule("s1", s1);"""),
    "bfs_hybrid": ("bfs.gt", ["parent"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(TWCE);
    SimpleGPUSchedule s2;
    s2.configDirection(PULL, BITMAP);
    s2.configFrontierCreation(UNFUSED_BITMAP);
    HybridGPUSchedule h1(INPUT_VERTEXSET_SIZE, 0.05, s1, s2);
    program->applyGPUSchedule("s1", h1);"""),
    "sssp_push_strict": ("sssp.gt", ["dist"], None),
    "sssp_push_vp_nodedup": ("sssp.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(VERTEX_BASED);
    s1.configDeduplication(DISABLED);
    program->applyGPUSchedule("s1", s1);"""),
    "sssp_pull": ("sssp.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configDirection(PULL);
    program->applyGPUSchedule("s1", s1);"""),
    "cc_push_etwc": ("cc.gt", ["IDs"], None),
    "cc_push_edge_only": ("cc.gt", ["IDs"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(EDGE_ONLY);
    program->applyGPUSchedule("s1", s1);"""),
    "bfs_fused_hybrid_strict": ("bfs.gt", ["parent"], """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    s1.configLoadBalance(STRICT);
    SimpleGPUSchedule s2;
    s2.configDirection(PULL, BITMAP);
    HybridGPUSchedule h1(INPUT_VERTEXSET_SIZE, 0.05, s1, s2);
    program->applyGPUSchedule("s1", h1);"""),
    "bfs_fused_wm_boolpull": ("bfs.gt", ["parent"], """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    s1.configLoadBalance(WM);
    SimpleGPUSchedule s2;
    s2.configDirection(PULL, BOOLMAP);
    HybridGPUSchedule h1(INPUT_VERTEXSET_SIZE, 0.02, s1, s2);
    program->applyGPUSchedule("s1", h1);"""),
    "sssp_fused_etwc": ("sssp.gt", ["dist"], """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    s1.configLoadBalance(ETWC);
    program->applyGPUSchedule("s1", s1);"""),
    "sssp_fused_vp_nodedup": ("sssp.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(VERTEX_BASED);
    s1.configDeduplication(DISABLED);
    s1.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s1", s1);"""),
    "cc_fused_cm": ("cc.gt", ["IDs"], """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    s1.configLoadBalance(CM);
    program->applyGPUSchedule("s1", s1);"""),
    "bfs_rounds": ("bfs_rounds.gt", ["parent", "seen", "info"], None),
    "bfs_rounds_fused": ("bfs_rounds.gt", ["parent", "seen", "info"], """
    SimpleGPUSchedule s0;
    s0.configKernelFusion(ENABLED);
    program->applyGPUSchedule("s0", s0);
    SimpleGPUSchedule s1;
    s1.configLoadBalance(STRICT);
    SimpleGPUSchedule s2;
    s2.configDirection(PULL, BITMAP);
    HybridGPUSchedule h1(INPUT_VERTEXSET_SIZE, 0.05, s1, s2);
    program->applyGPUSchedule("s1", h1);"""),
    "sssp_pq_strict_d64": ("sssp_pq.gt", ["dist"], None),
    "sssp_pq_etwc_d1": ("sssp_pq.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(ETWC);
    s1.configDelta(1);
    program->applyGPUSchedule("s1", s1);"""),
    "sssp_pq_cm_d4096_boolmap": ("sssp_pq.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(CM);
    s1.configDelta(4096);
    s1.configFrontierCreation(UNFUSED_BOOLMAP);
    program->applyGPUSchedule("s1", s1);"""),
    "sssp_pq_vp_d512_nodedup": ("sssp_pq.gt", ["dist"], """
    SimpleGPUSchedule s1;
    s1.configLoadBalance(VERTEX_BASED);
    s1.configDelta(512);
    s1.configDeduplication(DISABLED);
    program->applyGPUSchedule("s1", s1);"""),
    "pagerank_pull": ("pagerank.gt", ["old_rank"], None),
    "pagerank_push_blocked": ("pagerank.gt", ["old_rank"], """
    SimpleGPUSchedule s1;
    s1.configDirection(PUSH);
    s1.configLoadBalance(EDGE_ONLY, BLOCKED, 1000);
    program->applyGPUSchedule("s1", s1);"""),
    "pagerank_push_strict": ("pagerank.gt", ["old_rank"], """
    SimpleGPUSchedule s1;
    s1.configDirection(PUSH);
    s1.configLoadBalance(STRICT);
    program->applyGPUSchedule("s1", s1);"""),
}


def variant_source(name: str) -> str:
    fname, _, sched = VARIANTS[name]
    src = open(os.path.join(EXAMPLES, fname)).read()
    if sched is not None:
        src = src[:src.index("schedule:")] + "schedule:" + sched + "\n"
    return src


def build_examples(jobs: int = 8, force: bool = False) -> List[str]:
    """Compile every example variant into _gen/ (in parallel)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {n: ex.submit(build_only, variant_source(n), n, VARIANTS[n][1], None, force) for n in VARIANTS}
        return [f.result() for f in futs.values()]
