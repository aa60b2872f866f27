"""Lowering of a parsed program and its schedules to HIP C++ (the GPU Backend
Implementation section's code generation, for the supported subset).

What the analyses decide:

* Schedules: every labelled operator gets a gg_schedule built from the
  SimpleGPUSchedule / HybridGPUSchedule objects applied to its label (the
  defaults of the SimpleGPUSchedule table otherwise). They are compile-time
  constants of the generated code.
* Atomic insertion: an edge function run in the PUSH direction can be
  applied to one destination by many sources at once, so every write to a
  destination-indexed vector becomes an atomic: `min=` an atomic minimum, `+=`
  an atomic add, `=` a compare-and-swap when the `to` filter tests that same
  vector against a constant (the filter's check and the write become one
  CAS, which is also what makes applyModified's deduplication exact), else an
  atomic exchange. In the PULL direction each destination belongs to one lane
  and the writes stay plain; the lane stops scanning once the filter fails.
* Enqueue rewriting: applyModified(f, vec, true) puts a destination in the
  output frontier when its update changed `vec` (the CAS or minimum
  succeeded, the exchanged value differed).
* Frontier reuse (liveness): `delete frontier; frontier = output;` after an
  operator becomes the swap of the double-buffered frontier; nothing is
  allocated inside the loop.

The generated module defines one functor per (edge function, direction) and
per vertex function, and `gen_main`, the translated main function.
"""
from __future__ import annotations

from typing import Dict, List, Optional

from .lang import CompileError, Func, Program

CTYPE = {"int": "int32_t", "float": "float", "double": "double", "bool": "int32_t"}

LB = {"VERTEX_BASED": "GG_LB_VERTEX_BASED", "WM": "GG_LB_WM", "CM": "GG_LB_CM", "STRICT": "GG_LB_STRICT",
      "TWC": "GG_LB_TWC", "TWCE": "GG_LB_ETWC", "ETWC": "GG_LB_ETWC", "EDGE_ONLY": "GG_LB_EDGE_ONLY"}
CREATE = {"FUSED": "GG_CREATE_FUSED", "UNFUSED_BOOLMAP": "GG_CREATE_UNFUSED_BOOLMAP",
          "UNFUSED_BITMAP": "GG_CREATE_UNFUSED_BITMAP"}
DEDUP = {"MONOTONIC_COUNTERS": "GG_DEDUP_MONOTONIC_COUNTERS", "BITMAP": "GG_DEDUP_BITMAP",
         "BOOLMAP": "GG_DEDUP_BOOLMAP"}


# ---- schedules ------------------------------------------------------------------------------
def simple_default():
    return {"load_balance": "GG_LB_VERTEX_BASED", "edge_blocking": 0, "blocking_size": 1 << 20,
            "direction": "GG_PUSH", "pull_rep": "GG_REP_BOOLMAP", "frontier_creation": "GG_CREATE_FUSED",
            "dedup_enable": 1, "dedup_type": "GG_DEDUP_MONOTONIC_COUNTERS", "delta": 1, "kernel_fusion": 0}


def lower_schedules(prog: Program) -> Dict[str, dict]:
    """label -> {"hybrid", "threshold", "s1", "s2"} from the schedule section."""
    objs: Dict[str, dict] = {}
    out: Dict[str, dict] = {}
    for st in prog.schedule:
        if st[0] == "decl":
            _, kind, name, args = st
            if kind == "SimpleGPUSchedule":
                objs[name] = {"hybrid": 0, "threshold": 0.05, "s1": simple_default(), "s2": simple_default()}
            else:
                if len(args) != 4 or args[0][1] != "INPUT_VERTEXSET_SIZE":
                    raise CompileError("HybridGPUSchedule(INPUT_VERTEXSET_SIZE, threshold, s1, s2) expected")
                a, b = objs.get(args[2][1]), objs.get(args[3][1])
                if a is None or b is None:
                    raise CompileError("HybridGPUSchedule names an undeclared SimpleGPUSchedule")
                objs[name] = {"hybrid": 1, "threshold": float(args[1][1]), "s1": dict(a["s1"]), "s2": dict(b["s1"])}
        elif st[0] == "config":
            _, name, method, args = st
            if name not in objs:
                raise CompileError("schedule %r is not declared" % name)
            s = objs[name]["s1"]
            vals = [a[1] for a in args]
            if method == "configDirection":
                s["direction"] = "GG_PULL" if vals[0] == "PULL" else "GG_PUSH"
                if len(vals) > 1:
                    s["pull_rep"] = "GG_REP_BITMAP" if vals[1] == "BITMAP" else "GG_REP_BOOLMAP"
            elif method == "configLoadBalance":
                if vals[0] not in LB:
                    raise CompileError("unknown load balance %r" % vals[0])
                s["load_balance"] = LB[vals[0]]
                if vals[0] == "EDGE_ONLY" and len(vals) > 1 and vals[1] == "BLOCKED":
                    s["edge_blocking"] = 1
                    if len(vals) > 2:
                        s["blocking_size"] = int(vals[2])
                        if s["blocking_size"] < 1:
                            raise CompileError("blocking size must be >= 1")
            elif method == "configFrontierCreation":
                s["frontier_creation"] = CREATE[vals[0]]
            elif method == "configDeduplication":
                s["dedup_enable"] = 1 if vals[0] == "ENABLED" else 0
                if len(vals) > 1:
                    s["dedup_type"] = DEDUP[vals[1]]
            elif method == "configDelta":
                s["delta"] = int(vals[0])
            elif method == "configKernelFusion":
                s["kernel_fusion"] = 1 if vals[0] == "ENABLED" else 0
            else:
                raise CompileError("unknown schedule call %s" % method)
        else:
            _, label, name = st
            if name not in objs:
                raise CompileError("schedule %r is not declared" % name)
            out[label] = objs[name]
    return out


def float_literal(x: float) -> str:
    """C++ float literal (repr keeps a decimal point or an exponent)."""
    return repr(float(x)) + "f"


def sched_literal(s: Optional[dict]) -> str:
    if s is None:
        s = {"hybrid": 0, "threshold": 0.05, "s1": simple_default(), "s2": simple_default()}

    def simple(x):
        return "{%s, %d, %d, %s, %s, %s, %d, %s, %d, %d}" % (
            x["load_balance"], x["edge_blocking"], x["blocking_size"], x["direction"], x["pull_rep"],
            x["frontier_creation"], x["dedup_enable"], x["dedup_type"], x["delta"], x["kernel_fusion"])
    return "gg_schedule{%d, %s, %s, %s}" % (s["hybrid"], float_literal(s["threshold"]), simple(s["s1"]),
                                             simple(s["s2"]))


# ---- expressions --------------------------------------------------------------------------
class ExprGen:
    """C++ text of an expression in a function of the program; `names` maps
    the function's vertex parameters to C++ variables."""

    def __init__(self, prog: Program, names: Dict[str, str], weight: Optional[str] = None, host=False,
                 wide=False):
        # wide: integer vector elements and weights are read as int64_t, so
        # sums of a priority and a weight cannot wrap
        self.prog, self.names, self.weight, self.host, self.wide = prog, names, weight, host, wide

    def __call__(self, e) -> str:
        k = e[0]
        if k == "num":
            t = e[1]
            return t if ("." in t or "e" in t.lower()) else t
        if k == "bool":
            return "1" if e[1] else "0"
        if k == "id":
            n = e[1]
            if n in self.names:
                return self.names[n]
            if self.weight is not None and n == self.weight:
                return "(int64_t)w[e]" if self.wide else "(int32_t)w[e]"
            if n in self.prog.scalars:
                return "s_" + n
            raise CompileError("unknown name %r" % n)
        if k == "index":
            base = e[1]
            if base[0] != "id" or base[1] not in self.prog.vectors:
                raise CompileError("only vectors are indexed")
            if self.host:
                raise CompileError("main reads vector elements only through operators")
            if self.wide and self.prog.vectors[base[1]]["type"] in ("int", "bool"):
                return "(int64_t)vec_%s[%s]" % (base[1], self(e[2]))
            return "vec_%s[%s]" % (base[1], self(e[2]))
        if k == "bin":
            return "(%s %s %s)" % (self(e[2]), e[1], self(e[3]))
        if k == "un":
            return "(%s%s)" % (e[1], self(e[2]))
        if k == "method" and e[2] == "size" and e[1] == ("id", self.prog.vertices):
            return "(double)g.n"
        raise CompileError("unsupported expression %r" % (e,))


# ---- edge functions -------------------------------------------------------------------------
def _index_target(e, src: str, dst: str):
    """('dst'|'src', vector) for vec[dst] / vec[src]."""
    if e[0] != "index" or e[1][0] != "id" or e[2][0] != "id":
        raise CompileError("an edge function assigns to vec[src] or vec[dst]")
    who = {src: "src", dst: "dst"}.get(e[2][1])
    if who is None:
        raise CompileError("an edge function indexes vectors with its src or dst parameter")
    return who, e[1][1]


def _filter_cas(prog: Program, filt: Optional[Func], vec: str):
    """If the filter is `output = vec[v] == C;` return C's text (the CAS's expected value)."""
    if filt is None or len(filt.body) != 1:
        return None
    st = filt.body[0]
    if st[0] != "assign" or st[1] != "=" or st[2] != ("id", filt.result[0]):
        return None
    e = st[3]
    if e[0] == "bin" and e[1] == "==" and e[2][0] == "index" and e[2][1] == ("id", vec) \
            and e[2][2] == ("id", filt.params[0][0]):
        c = e[3]
        if c[0] == "num" or (c[0] == "un" and c[1] == "-" and c[2][0] == "num"):
            return ExprGen(prog, {})(c)
    return None


def edge_functor(prog: Program, f: Func, direction: str, filt: Optional[Func], tracked: Optional[str],
                 cname: str, notes: List[str]) -> str:
    """One functor for edge function f applied in `direction` ('push'/'pull')
    from a frontier to destinations passing `filt`, tracking `tracked`."""
    if len(f.params) not in (2, 3):
        raise CompileError("edge function %s takes (src, dst[, weight])" % f.name)
    src, dst = f.params[0][0], f.params[1][0]
    weight = f.params[2][0] if len(f.params) == 3 else None
    g = ExprGen(prog, {src: "u", dst: "v"}, weight)
    vecs = sorted(prog.vectors)
    members = "".join("    %s *vec_%s;\n" % (CTYPE[prog.vectors[v]["type"]], v) for v in vecs)
    members += "".join("    double s_%s;\n" % s for s in sorted(prog.scalars))
    members += "    const uint32_t *w;\n"
    fcond = "true"
    if filt is not None:
        fv = filt.params[0][0]
        fg = ExprGen(prog, {fv: "v"})
        body = filt.body
        if len(body) != 1 or body[0][0] != "assign" or body[0][2] != ("id", filt.result[0]):
            raise CompileError("a filter function is `output = <expression>;`")
        fcond = fg(body[0][3])
    lines = []
    modified = []
    cas_used = False
    for st in f.body:
        if st[0] != "assign":
            raise CompileError("edge function %s: only assignments are supported" % f.name)
        op, lhs, rhs = st[1], st[2], st[3]
        who, vec = _index_target(lhs, src, dst)
        if who != "dst":
            raise CompileError("edge function %s writes %s[%s]: only destination writes are supported"
                               % (f.name, vec, src))
        ty = prog.vectors[vec]["type"]
        ct = CTYPE[ty]
        val = g(rhs)
        mod = "m_%d" % len(modified)
        modified.append((vec, mod))
        if direction == "pull":
            if op == "=":
                lines.append("const %s nv_%s = (%s)(%s); const bool %s = vec_%s[v] != nv_%s; vec_%s[v] = nv_%s;"
                             % (ct, mod, ct, val, mod, vec, mod, vec, mod))
            elif op == "min=":
                lines.append("const %s nv_%s = (%s)(%s); const bool %s = nv_%s < vec_%s[v]; if (%s) vec_%s[v] = nv_%s;"
                             % (ct, mod, ct, val, mod, mod, vec, mod, vec, mod))
            else:
                lines.append("vec_%s[v] += (%s)(%s); const bool %s = true;" % (vec, ct, val, mod))
            continue
        # PUSH: atomic insertion
        if op == "min=":
            if ty != "int":
                raise CompileError("min= on a %s vector is not supported in PUSH (int vectors only)" % ty)
            lines.append("const int32_t nv_%s = (int32_t)(%s); const bool %s = nv_%s < vec_%s[v] && "
                         "atomic_min_i32(&vec_%s[v], nv_%s) > nv_%s;" % (mod, val, mod, mod, vec, vec, mod, mod))
            notes.append("%s: %s[dst] min= ... -> atomic minimum (PUSH)" % (f.name, vec))
        elif op == "+=":
            fn = {"float": "atomic_add_f32", "double": "atomic_add_f64", "int": "atomic_add_i32"}[ty]
            lines.append("(void)%s(&vec_%s[v], (%s)(%s)); const bool %s = true;" % (fn, vec, ct, val, mod))
            notes.append("%s: %s[dst] += ... -> atomic add (PUSH)" % (f.name, vec))
        else:
            if ty != "int":
                raise CompileError("= on a %s vector is not supported in PUSH (int vectors only)" % ty)
            expected = _filter_cas(prog, filt, vec)
            if expected is not None:
                lines.append("const bool %s = atomic_cas_i32(&vec_%s[v], %s, (int32_t)(%s)) == %s;"
                             % (mod, vec, expected, val, expected))
                notes.append("%s: filter %s(v) tests %s[v] == %s and the function writes %s[dst] -> one "
                             "compare-and-swap (PUSH)" % (f.name, filt.name, vec, expected, vec))
                cas_used = True
            else:
                lines.append("const int32_t nv_%s = (int32_t)(%s); const bool %s = __hip_atomic_exchange("
                             "&vec_%s[v], nv_%s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != nv_%s;"
                             % (mod, val, mod, vec, mod, mod))
                notes.append("%s: %s[dst] = ... -> atomic exchange (PUSH)" % (f.name, vec))
    if direction == "pull":
        notes.append("%s: PULL -> plain writes (one lane per destination), early exit when %s fails"
                     % (f.name, filt.name if filt else "the filter"))
    if tracked is not None:
        tm = [m for vec, m in modified if vec == tracked]
        if not tm:
            raise CompileError("applyModified tracks %s, which %s does not write" % (tracked, f.name))
        ret = "(%s) ? v : -1" % " || ".join(tm)
    else:
        ret = "-1"
    body = "\n        ".join(lines)
    if direction == "push":
        return """struct %s {
%s    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    using Pre = int;
    __device__ __forceinline__ Pre load(int, int, int) const { return 0; }
    __device__ __forceinline__ int apply(int u, int v, int e, Pre) const {
        if (!(%s)) return -1;
        %s
        return %s;
    }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, 0); }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};
""" % (cname, members, fcond, body, ret)
    return """struct %s {
%s    __device__ __forceinline__ bool active(int v) const { return %s; }
    __device__ __forceinline__ bool done(int v) const { return !(%s); }
    using Pre = int;
    __device__ __forceinline__ Pre load(int, int, int) const { return 0; }
    __device__ __forceinline__ int apply(int u, int v, int e, Pre) const {
        %s
        return %s;
    }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, 0); }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};
""" % (cname, members, fcond, fcond, body, ret)


def pq_edge_functor(prog: Program, f: Func, pq: str, cname: str, notes: List[str]) -> str:
    """Functor for edges.from(frontier).applyUpdatePriority(f): f's local
    variables, then pq.updatePriorityMin(dst, value) lowered to an atomic
    minimum on the priority vector that also sorts the destination into the
    ready set (current bucket) or the far queue (a later bucket)."""
    if len(f.params) not in (2, 3):
        raise CompileError("edge function %s takes (src, dst[, weight])" % f.name)
    src, dst = f.params[0][0], f.params[1][0]
    weight = f.params[2][0] if len(f.params) == 3 else None
    names = {src: "u", dst: "v"}
    members = "".join("    %s *vec_%s;\n" % (CTYPE[prog.vectors[v]["type"]], v) for v in sorted(prog.vectors))
    members += "".join("    double s_%s;\n" % s for s in sorted(prog.scalars))
    members += "    const uint32_t *w;\n    gen::PQView pq;\n"
    lines, ups = [], []
    for st in f.body:
        if st[0] == "var" and st[2][0] == "scalar" and st[3] is not None:
            lname = "l_" + st[1]
            lines.append("const int64_t %s = (int64_t)(%s);" % (lname, ExprGen(prog, names, weight, wide=True)(st[3])))
            names[st[1]] = lname
        elif (st[0] == "expr" and st[1][0] == "method" and st[1][1] == ("id", pq)
              and st[1][2] == "updatePriorityMin"):
            args = st[1][3]
            if len(args) != 2 or args[0] != ("id", dst):
                raise CompileError("%s.updatePriorityMin(%s, value) updates the destination" % (pq, dst))
            k = len(ups)
            lines.append("bool tf_%d; const bool n_%d = gen::pq_update_min(pq, v, (long long)(%s), tf_%d);"
                         % (k, k, ExprGen(prog, names, weight, wide=True)(args[1]), k))
            lines.append("wave_append(pq.farq, pq.farc, pq.far_cap, pq.flags + 1, tf_%d, v);" % k)
            ups.append("n_%d" % k)
        else:
            raise CompileError("edge function %s: local variables and %s.updatePriorityMin(...) are supported "
                               "under applyUpdatePriority" % (f.name, pq))
    if not ups:
        raise CompileError("edge function %s does not call %s.updatePriorityMin" % (f.name, pq))
    notes.append("%s: %s.updatePriorityMin -> atomic minimum on the priority vector, bucket test, ready set "
                 "or far queue (PUSH)" % (f.name, pq))
    return """struct %s {
%s    __device__ __forceinline__ bool active(int) const { return true; }
    __device__ __forceinline__ bool done(int) const { return false; }
    using Pre = int;
    __device__ __forceinline__ Pre load(int, int, int) const { return 0; }
    __device__ __forceinline__ int apply(int u, int v, int e, Pre) const {
        %s
        return (%s) ? v : -1;
    }
    __device__ __forceinline__ int edge(int u, int v, int e) const { return apply(u, v, e, 0); }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ void flush() const {}
};
""" % (cname, members, "\n        ".join(lines), " || ".join(ups))


def vertex_functor(prog: Program, f: Func, cname: str) -> str:
    if len(f.params) != 1:
        raise CompileError("vertex function %s takes (v)" % f.name)
    v = f.params[0][0]
    g = ExprGen(prog, {v: "v"})
    members = "".join("    %s *vec_%s;\n" % (CTYPE[prog.vectors[x]["type"]], x) for x in sorted(prog.vectors))
    members += "".join("    double s_%s;\n" % s for s in sorted(prog.scalars))
    lines = []
    for st in f.body:
        if st[0] != "assign" or st[2][0] != "index" or st[2][2] != ("id", v):
            raise CompileError("vertex function %s: only assignments to vec[%s] are supported" % (f.name, v))
        vec = st[2][1][1]
        ct = CTYPE[prog.vectors[vec]["type"]]
        val = g(st[3])
        if st[1] == "=":
            lines.append("vec_%s[v] = (%s)(%s);" % (vec, ct, val))
        elif st[1] == "+=":
            lines.append("vec_%s[v] += (%s)(%s);" % (vec, ct, val))
        else:
            lines.append("{ const %s nv = (%s)(%s); if (nv < vec_%s[v]) vec_%s[v] = nv; }" % (ct, ct, val, vec, vec))
    return """struct %s {
%s    __device__ __forceinline__ void operator()(int v) const {
        %s
    }
};
""" % (cname, members, "\n        ".join(lines))


# ---- main ---------------------------------------------------------------------------------------
class MainGen:
    def __init__(self, prog: Program, scheds: Dict[str, dict], notes: List[str]):
        self.prog, self.scheds, self.notes = prog, scheds, notes
        self.functors: Dict[str, str] = {}   # C++ name -> definition
        self.fused_kernels: List[str] = []   # persistent kernels of fused loops
        self.pq_made: Dict[str, bool] = {}     # priority queues created in main
        self.host_vars: Dict[str, str] = {}
        self.frontiers: Dict[str, str] = {}  # program name -> "fs"
        self.labels_used: List[str] = []
        self.out: List[str] = []
        self.uses_edge_only = False
        self.uses_pull = False
        self.needs_ids = False
        self.no_dedup = False

    def hexpr(self, e) -> str:
        k = e[0]
        if k == "id" and e[1] in self.host_vars:
            return self.host_vars[e[1]]
        if k == "call" and e[1] == "atoi":
            a = e[2][0]
            if a[0] != "index" or a[1] != ("id", "argv") or a[2][0] != "num":
                raise CompileError("atoi takes argv[k]")
            k_ = int(a[2][1])
            if k_ < 2:
                raise CompileError("argv[0] is the program and argv[1] the graph")
            return "arg(%d)" % (k_ - 2)
        if k == "bin":
            return "(%s %s %s)" % (self.hexpr(e[2]), e[1], self.hexpr(e[3]))
        if k == "un":
            return "(%s%s)" % (e[1], self.hexpr(e[2]))
        if k == "method" and e[2] == "size" and e[1] == ("id", self.prog.vertices):
            return "(int64_t)g.n"
        return ExprGen(self.prog, {}, host=True)(e)

    def init_list(self, with_w: bool) -> str:
        items = ["vec_%s.p" % v for v in sorted(self.prog.vectors)] + ["s_%s" % s for s in sorted(self.prog.scalars)]
        if with_w:
            items.append("g.w")
        return "{" + ", ".join(items) + "}"

    def edge_functor_for(self, fname: str, direction: str, filt: Optional[str], tracked: Optional[str]) -> str:
        f = self.prog.funcs.get(fname)
        if f is None:
            raise CompileError("unknown function %s" % fname)
        ff = self.prog.funcs.get(filt) if filt else None
        if filt and ff is None:
            raise CompileError("unknown filter %s" % filt)
        cname = "E_%s_%s%s%s" % (fname, direction, "_" + filt if filt else "", "_" + tracked if tracked else "")
        if cname not in self.functors:
            self.functors[cname] = edge_functor(self.prog, f, direction, ff, tracked, cname, self.notes)
        return cname

    def vertex_functor_for(self, fname: str) -> str:
        f = self.prog.funcs.get(fname)
        if f is None:
            raise CompileError("unknown function %s" % fname)
        cname = "V_%s" % fname
        if cname not in self.functors:
            self.functors[cname] = vertex_functor(self.prog, f, cname)
        return cname

    def sched(self, label: Optional[str]) -> str:
        s = self.scheds.get(label) if label else None
        name = "sch_%s" % (label or "default")
        if name not in self.labels_used:
            self.labels_used.append(name)
            self.out.insert(0, "    const gg_schedule %s = %s;" % (name, sched_literal(s)))
            for x in ([s["s1"], s["s2"]] if s and s["hybrid"] else [s["s1"]] if s else []):
                if x["load_balance"] == "GG_LB_EDGE_ONLY":
                    self.uses_edge_only = True
                if x["direction"] == "GG_PULL":
                    self.uses_pull = True
                if x["frontier_creation"] == "GG_CREATE_FUSED" and not x["dedup_enable"]:
                    self.no_dedup = True
        return name

    def emit(self, text: str, depth: int):
        self.out.append("    " * depth + text)

    def stmts(self, body, depth: int):
        i = 0
        while i < len(body):
            st = body[i]
            k = st[0]
            if k == "var":
                _, name, ty, init, label, line = st
                if ty[0] == "scalar":
                    cname = "h_" + name
                    self.host_vars[name] = cname
                    self.emit("int64_t %s = %s;" % (cname, self.hexpr(init) if init is not None else "0"), depth)
                elif ty[0] == "vertexset":
                    if init is None:
                        raise CompileError("line %d: a vertexset variable needs an initial value" % line)
                    if init[0] == "new":
                        if self.frontiers:
                            raise CompileError("line %d: one frontier variable per program is supported" % line)
                        self.frontiers[name] = "fs"
                        if len(init[2]) != 1:
                            raise CompileError("line %d: new vertexset{Vertex}(size) takes one argument" % line)
                        arg = init[2][0]
                        if arg == ("num", "0"):
                            self.emit("fs.count = 0;", depth)
                        elif arg[0] == "method" and arg[2] == "size" and arg[1] == ("id", self.prog.vertices):
                            self.emit("hipLaunchKernelGGL(gen::k_gen_iota, dim3(blocks_for(g.n, kBlock, 8192)), "
                                      "dim3(kBlock), 0, c.s, fs.queue(), g.n);", depth)
                            self.emit("GG_CHECK_LAUNCH();", depth)
                            self.emit("fs.count = g.n;", depth)
                        else:
                            raise CompileError("line %d: new vertexset(0) or new vertexset(vertices.size())" % line)
                    else:
                        self.frontier_op(name, init, label, line, depth, body, i)
                        i += 2  # the delete / reassignment that follow are the frontier swap
                else:
                    raise CompileError("line %d: unsupported variable type %r" % (line, ty))
            elif k == "assign":
                _, op, lhs, rhs, label, line = st
                if lhs[0] == "id" and lhs[1] in self.prog.pqs:
                    self.pq_create(lhs[1], rhs, line, depth)
                elif lhs[0] == "id" and lhs[1] in self.host_vars and op in ("=", "+="):
                    self.emit("%s %s %s;" % (self.host_vars[lhs[1]], op, self.hexpr(rhs)), depth)
                elif lhs[0] == "index" and lhs[1][0] == "id" and lhs[1][1] in self.prog.vectors and op == "=":
                    vec = lhs[1][1]
                    ct = CTYPE[self.prog.vectors[vec]["type"]]
                    self.emit("gen::set_one<%s>(c, vec_%s.p, g.n, (int64_t)(%s), (%s)(%s));"
                              % (ct, vec, self.hexpr(lhs[2]), ct, self.hexpr(rhs)), depth)
                else:
                    raise CompileError("line %d: unsupported assignment in main" % line)
            elif k == "expr":
                _, e, label, line = st
                self.call(e, label, line, depth)
            elif k == "while" and self.pq_cond(st[1]) is not None:
                self.pq_loop(self.pq_cond(st[1]), st[2], st[4], depth)
            elif k == "while":
                _, cond, wbody, label, line = st
                if not (cond[0] == "bin" and cond[1] == "!=" and cond[3] == ("num", "0") and cond[2][0] == "method"
                        and cond[2][2] == "getVertexSetSize" and cond[2][1][0] == "id"
                        and cond[2][1][1] in self.frontiers):
                    raise CompileError("line %d: while (frontier.getVertexSetSize() != 0) is the supported loop" % line)
                ops = [j for j, x in enumerate(wbody) if x[0] == "var" and x[2] == ("vertexset",)]
                op = wbody[ops[0]] if len(ops) == 1 else None
                wsched = self.scheds.get(label) if label else None
                osched = self.scheds.get(op[4]) if op is not None and op[4] else None
                if (wsched and wsched["s1"]["kernel_fusion"]) or (osched and osched["s1"]["kernel_fusion"]):
                    if op is None or op[3] is None:
                        raise CompileError("line %d: a fused loop holds one frontier operator" % line)
                    self.fused_while(wbody, ops[0], op[4] if osched else label, line, depth)
                else:
                    self.emit("while (fs.count > 0) {", depth)
                    self.stmts(wbody, depth + 1)
                    self.emit("}", depth)
            elif k == "for":
                _, var, lo, hi, fbody, label, line = st
                cname = "h_" + var
                self.host_vars[var] = cname
                self.emit("for (int64_t %s = %s; %s < %s; %s++) {" % (cname, self.hexpr(lo), cname,
                                                                    self.hexpr(hi), cname), depth)
                self.stmts(fbody, depth + 1)
                self.emit("}", depth)
            elif k == "delete":
                pass  # storage is released when main returns (and reused by the frontier swap)
            else:
                raise CompileError("unsupported statement %r" % (k,))
            i += 1

    def blocked(self, label) -> bool:
        s = self.scheds.get(label) if label else None
        return bool(s) and any(x["edge_blocking"] for x in ([s["s1"], s["s2"]] if s["hybrid"] else [s["s1"]]))

    def pq_create(self, pq, rhs, line, depth):
        """pq = new priority_queue{Vertex}(int)(priority_vector, start_vertex)"""
        if rhs[0] != "new" or rhs[1][0] != "pq" or len(rhs[2]) != 2 or rhs[2][0][0] != "id" \
                or rhs[2][0][1] not in self.prog.vectors:
            raise CompileError("line %d: %s = new priority_queue{Vertex}(int)(vector, start_vertex)" % (line, pq))
        vec = rhs[2][0][1]
        if self.prog.vectors[vec]["type"] != "int":
            raise CompileError("line %d: the priority vector %s must hold int" % (line, vec))
        if pq in self.pq_made:
            raise CompileError("line %d: %s is created once" % (line, pq))
        self.pq_made[pq] = True
        self.emit("gen::PQState pq_%s;" % pq, depth)
        self.emit("pq_%s.prio = vec_%s.p;" % (pq, vec), depth)
        self.emit("pq_%s.start = (int64_t)(%s);" % (pq, self.hexpr(rhs[2][1])), depth)
        self.emit("pq_%s.n = g.n;" % pq, depth)

    def pq_cond(self, cond):
        """The queue of `while (pq.finished() == false)` (or `!pq.finished()`), else None."""
        def fin(e):
            return e[0] == "method" and e[2] == "finished" and e[1][0] == "id" and e[1][1] in self.prog.pqs
        if cond[0] == "bin" and cond[1] == "==" and fin(cond[2]) and cond[3] == ("bool", False):
            return cond[2][1][1]
        if cond[0] == "un" and cond[1] == "!" and fin(cond[2]):
            return cond[2][1][1]
        return None

    def pq_loop(self, pq, body, line, depth):
        """while (pq.finished() == false): frontier = pq.dequeue_ready_set();
        edges.from(frontier).applyUpdatePriority(f); delete frontier;"""
        if pq not in self.pq_made:
            raise CompileError("line %d: %s is used before it is created" % (line, pq))
        ok = (len(body) == 3 and body[0][0] == "var" and body[0][2] == ("vertexset",)
              and body[0][3] is not None and body[0][3][0] == "method" and body[0][3][2] == "dequeue_ready_set"
              and body[0][3][1] == ("id", pq) and body[1][0] == "expr" and body[2][0] == "delete"
              and body[2][1] == body[0][1])
        if not ok:
            raise CompileError("line %d: the loop of %s holds `var f : vertexset{..} = %s.dequeue_ready_set();`, "
                               "`edges.from(f).applyUpdatePriority(update);` and `delete f;`" % (line, pq, pq))
        fname = body[0][1]
        e, label = body[1][1], body[1][2]
        if not (e[0] == "method" and e[2] == "applyUpdatePriority" and len(e[3]) == 1 and e[3][0][0] == "id"
                and e[1][0] == "method" and e[1][2] == "from" and e[1][1] == ("id", self.prog.edges["name"])
                and e[1][3] == [("id", fname)]):
            raise CompileError("line %d: expected %s.from(%s).applyUpdatePriority(update)"
                               % (body[1][-1], self.prog.edges["name"], fname))
        if self.frontiers and fname not in self.frontiers:
            raise CompileError("line %d: one frontier variable per program is supported" % line)
        self.frontiers[fname] = "fs"
        udf = self.prog.funcs.get(e[3][0][1])
        if udf is None:
            raise CompileError("unknown function %s" % e[3][0][1])
        if len(udf.params) == 3 and not self.prog.edges["weighted"]:
            raise CompileError("%s takes a weight but the edgeset is unweighted" % udf.name)
        s = self.scheds.get(label) if label else None
        for x in ([s["s1"], s["s2"]] if s and s["hybrid"] else [s["s1"]] if s else []):
            if x["direction"] != "GG_PUSH" or x["kernel_fusion"]:
                raise CompileError("line %d: applyUpdatePriority runs unfused PUSH steps" % line)
        delta = s["s1"]["delta"] if s else 1
        sname = self.sched(label)
        cname = "P_%s_%s" % (udf.name, pq)
        if cname not in self.functors:
            self.functors[cname] = pq_edge_functor(self.prog, udf, pq, cname, self.notes)
        init = self.init_list(True)[:-1] + ", gen::pq_view(pq_%s)}" % pq
        self.emit("gen::pq_start(c, *ws, fs, pq_%s, %d);" % (pq, delta), depth)
        self.emit("while (gen::pq_next(c, *ws, fs, pq_%s, iter)) {" % pq, depth)
        self.emit("    const gg_simple_schedule &sc = pick(%s, fs.count, g.n);" % sname, depth)
        self.emit("    gen::frontier_step(c, g, *ws, fs, sc, %s%s, ++iter);" % (cname, init), depth)
        self.emit("}", depth)
        self.notes.append("priority queue %s: buckets of width %d (configDelta), ready set in the frontier, "
                          "later buckets in a far queue" % (pq, delta))

    def dexpr(self, e) -> str:
        """A scalar expression inside a fused loop: hoisted locals of main and literals."""
        k = e[0]
        if k == "num":
            return e[1]
        if k == "bool":
            return "1" if e[1] else "0"
        if k == "id" and e[1] in self.host_vars:
            return self.host_vars[e[1]]
        if k == "bin":
            return "(%s %s %s)" % (self.dexpr(e[2]), e[1], self.dexpr(e[3]))
        if k == "un":
            return "(%s%s)" % (e[1], self.dexpr(e[2]))
        raise CompileError("inside a fused loop a scalar statement reads main's local variables and literals "
                           "only (%r)" % (e,))

    def fused_while(self, wbody, i_op, label, line, depth):
        """A fused loop (the GPU Backend section's kernel fusion): one generated
        persistent kernel runs the loop; main's local variables the body uses are
        hoisted to device memory (copied in before the launch, out after); scalar
        statements run in every lane alike, vertices.apply over the grid between
        grid barriers, the operator through the runtime's fused step."""
        op = wbody[i_op]
        pre, post = wbody[:i_op], wbody[i_op + 3:]
        if not pre and not post:
            # the operator and the swap alone: the runtime's fused loop kernel
            self.frontier_op(op[1], op[3], label, op[5], depth, wbody, i_op, fused=True)
            self.notes.append("while loop at line %d: kernel fusion -> one persistent launch for every round"
                              % line)
            return
        hoisted: List[str] = []
        applies: List[str] = []
        code_pre: List[str] = []
        code_post: List[str] = []

        def use(name):
            if name not in hoisted:
                hoisted.append(name)

        def walk(e):
            if isinstance(e, tuple):
                if e[0] == "id" and e[1] in self.host_vars:
                    use(e[1])
                for x in e[1:]:
                    walk(x)

        for where, stmts_, code in (("pre", pre, code_pre), ("post", post, code_post)):
            for st in stmts_:
                if st[0] == "assign" and st[2][0] == "id" and st[2][1] in self.host_vars and st[1] in ("=", "+="):
                    use(st[2][1])
                    walk(st[3])
                    code.append("%s %s %s;" % (self.host_vars[st[2][1]], st[1], self.dexpr(st[3])))
                elif (st[0] == "expr" and st[1][0] == "method" and st[1][2] == "apply"
                      and st[1][1] == ("id", self.prog.vertices)):
                    cname = self.vertex_functor_for(st[1][3][0][1])
                    k = len(applies)
                    applies.append(cname)
                    if where == "pre":
                        code.append("gen::fused_vertices(a.g.n, vf%d, s.t);" % k)
                        code.append("if (!grid_sync(s.bar)) break;")
                    else:
                        code.append("if (!grid_sync(s.bar)) break;")
                        code.append("gen::fused_vertices(a.g.n, vf%d, s.t);" % k)
                elif st[0] == "delete":
                    raise CompileError("line %d: in a fused loop `delete` belongs to the frontier swap" % st[-1])
                else:
                    raise CompileError("line %d: this statement cannot run inside a fused loop (scalar "
                                       "assignments, vertices.apply and the frontier operator can)" % st[-1])
        # the operator (checks its form and the swap that follows it) and its template arguments
        out_name = op[1]
        kid = len(self.fused_kernels)
        lb, dd, s2, th = self.fused_params(label, op[5])
        push, pull = self.frontier_op(out_name, op[3], label, op[5], depth, wbody, i_op, fused=None)
        kname = "k_fused_%d" % kid
        params = ["gen::GenFusedArgs a", "%s fp" % push, "%s fl" % pull, "int64_t *hoist"]
        params += ["%s vf%d" % (cn, k) for k, cn in enumerate(applies)]
        body = ["    gen::FusedLoopState s = gen::fused_begin(a);"]
        body += ["    int64_t %s = hoist[%d];" % (self.host_vars[h], j) for j, h in enumerate(hoisted)]
        body += ["    for (;;) {",
                 "        const int cnt = gen::fused_round_head(a, s);",
                 "        if (cnt < 0) break;"]
        body += ["        " + x for x in code_pre]
        body += ["        if (!gen::fused_step<%s, %s, %d>(a, fp, fl, s, cnt)) break;" % (lb, dd, s2)]
        body += ["        " + x for x in code_post]
        body += ["        if (!gen::fused_round_tail(s)) break;", "    }", "    gen::fused_end(a, s);"]
        if hoisted:
            body += ["    if (blockIdx.x == 0 && threadIdx.x == 0) {"]
            body += ["        hoist[%d] = %s;" % (j, self.host_vars[h]) for j, h in enumerate(hoisted)]
            body += ["    }"]
        self.fused_kernels.append("__global__ __launch_bounds__(kBlock) void %s(%s) {\n%s\n}\n"
                                  % (kname, ", ".join(params), "\n".join(body)))
        nh = max(len(hoisted), 1)
        init = self.init_list(True)
        host = ["if (fs.count > 0) {",
                "    DevBuf<int64_t> hoist;",
                "    hoist.ensure(%d);" % nh,
                "    int64_t hh[%d] = {%s};" % (nh, ", ".join(self.host_vars[h] for h in hoisted) or "0"),
                "    GG_HIP(hipMemcpyAsync(hoist.p, hh, sizeof(hh), hipMemcpyHostToDevice, c.s));",
                "    GG_HIP(hipStreamSynchronize(c.s));",
                "    const void *kern = (const void *)%s;" % kname,
                "    gen::FusedLaunch L = gen::fused_prepare(c, G, g, *ws, fs, %s, kern, %s, iter);"
                % (float_literal(th), "true" if lb == "GG_LB_STRICT" else "false"),
                "    %s fp%s;" % (push, init),
                "    %s fl%s;" % (pull, init),
                "    int64_t *hp = hoist.p;"]
        host += ["    %s vf%d%s;" % (cn, k, self.init_list(False)) for k, cn in enumerate(applies)]
        host += ["    void *args[] = {%s};" % ", ".join(["&L.a", "&fp", "&fl", "&hp"] +
                                                      ["&vf%d" % k for k in range(len(applies))]),
                 "    launch_cooperative(c, kern, L.blocks, args);",
                 "    gen::fused_complete(c, *ws, fs, iter);",
                 "    GG_HIP(hipMemcpyAsync(hh, hoist.p, sizeof(hh), hipMemcpyDeviceToHost, c.s));",
                 "    GG_HIP(hipStreamSynchronize(c.s));"]
        host += ["    %s = hh[%d];" % (self.host_vars[h], j) for j, h in enumerate(hoisted)]
        host += ["}"]
        for x in host:
            self.emit(x, depth)
        self.notes.append("while loop at line %d: kernel fusion -> %s, one persistent launch for every round%s"
                          % (line, kname, "; hoisted to device memory: " + ", ".join(hoisted) if hoisted else ""))

    def frontier_op(self, out_name, e, label, line, depth, body, i, fused=False):
        # edges.from(F)[.to(FILT)].applyModified(U, VEC, true)
        if e[0] != "method" or e[2] != "applyModified":
            raise CompileError("line %d: a frontier operator is edges.from(f)[.to(g)].applyModified(...)" % line)
        args = e[3]
        if len(args) != 3 or args[0][0] != "id" or args[1][0] != "id":
            raise CompileError("line %d: applyModified(function, vector, true)" % line)
        udf, tracked = args[0][1], args[1][1]
        base = e[1]
        filt = None
        if base[0] == "method" and base[2] == "to":
            filt = base[3][0][1]
            base = base[1]
        if not (base[0] == "method" and base[2] == "from" and base[1] == ("id", self.prog.edges["name"])):
            raise CompileError("line %d: expected %s.from(frontier)" % (line, self.prog.edges["name"]))
        fr = base[3][0]
        if fr[0] != "id" or fr[1] not in self.frontiers:
            raise CompileError("line %d: the operator's input is not the frontier variable" % line)
        # liveness: the output must replace the input frontier right after the operator
        rest = body[i + 1:i + 3]
        ok = (len(rest) == 2 and rest[0][0] == "delete" and rest[0][1] == fr[1] and rest[1][0] == "assign"
              and rest[1][1] == "=" and rest[1][2] == ("id", fr[1]) and rest[1][3] == ("id", out_name))
        if not ok:
            raise CompileError("line %d: after the operator, `delete %s; %s = %s;` is required (the output "
                               "frontier replaces the input; its buffer is reused)" % (line, fr[1], fr[1], out_name))
        self.notes.append("frontier %s: `delete %s; %s = %s;` -> double-buffer swap, no allocation in the loop"
                          % (fr[1], fr[1], fr[1], out_name))
        if self.blocked(label):
            raise CompileError("line %d: EdgeBlocking applies when every edge is processed (edges.apply), "
                               "not to a frontier operator" % line)
        sname = self.sched(label)
        push = self.edge_functor_for(udf, "push", filt, tracked)
        pull = self.edge_functor_for(udf, "pull", filt, tracked)
        w = self.prog.edges["weighted"]
        if w is False and any(p for p in self.prog.funcs[udf].params[2:]):
            raise CompileError("line %d: %s takes a weight but the edgeset is unweighted" % (line, udf))
        if fused is None:
            return push, pull
        if fused:
            lb, dd, s2, th = self.fused_params(label, line)
            self.emit("gen::fused_loop<%s, %s, %d>(c, G, g, *ws, fs, %s, %s%s, %s%s, iter);"
                      % (lb, dd, s2, float_literal(th), push, self.init_list(True), pull, self.init_list(True)),
                      depth)
            return
        self.emit("{", depth)
        self.emit("    const gg_simple_schedule &sc = pick(%s, fs.count, g.n);" % sname, depth)
        self.emit("    if (sc.direction == GG_PUSH) gen::frontier_step(c, g, *ws, fs, sc, %s%s, ++iter);"
                  % (push, self.init_list(True)), depth)
        self.emit("    else gen::frontier_step(c, g, *ws, fs, sc, %s%s, ++iter);" % (pull, self.init_list(True)), depth)
        self.emit("}", depth)

    def fused_params(self, label, line):
        """Template arguments of gen::fused_loop for the operator's schedule."""
        s = self.scheds.get(label) if label else None
        s1 = s["s1"] if s else simple_default()
        if s1["direction"] != "GG_PUSH" or s1["frontier_creation"] != "GG_CREATE_FUSED":
            raise CompileError("line %d: a fused loop starts with PUSH steps that build queues (FUSED creation)"
                               % line)
        if s1["load_balance"] not in ("GG_LB_VERTEX_BASED", "GG_LB_WM", "GG_LB_CM", "GG_LB_STRICT", "GG_LB_ETWC"):
            raise CompileError("line %d: a fused loop runs VERTEX_BASED, WM, CM, STRICT or ETWC" % line)
        if not s1["dedup_enable"]:
            dd = "kDedupNone"
        elif s1["dedup_type"] == "GG_DEDUP_MONOTONIC_COUNTERS":
            dd = "kDedupMonotonic"
        else:
            raise CompileError("line %d: a fused loop deduplicates with monotonic counters" % line)
        s2, th = 0, 0.0
        if s and s["hybrid"]:
            if s["s2"]["direction"] != "GG_PULL":
                raise CompileError("line %d: a fused hybrid loop switches to a PULL step" % line)
            s2 = 2 if s["s2"]["pull_rep"] == "GG_REP_BITMAP" else 1
            th = s["threshold"]
        return s1["load_balance"], dd, s2, th

    def call(self, e, label, line, depth):
        if e[0] != "method":
            raise CompileError("line %d: unsupported expression statement" % line)
        target, name, args = e[1], e[2], e[3]
        if name == "addVertex" and target[0] == "id" and target[1] in self.frontiers:
            self.emit("gen::add_vertex(c, fs, g.n, (int64_t)(%s));" % self.hexpr(args[0]), depth)
        elif name == "apply" and target == ("id", self.prog.vertices):
            cname = self.vertex_functor_for(args[0][1])
            self.emit("gen::vertices_apply(c, g.n, %s%s);" % (cname, self.init_list(False)), depth)
        elif name == "apply" and target == ("id", self.prog.edges["name"]) and self.blocked(label):
            s1 = self.scheds[label]["s1"]
            if s1["direction"] != "GG_PUSH" or self.scheds[label]["hybrid"]:
                raise CompileError("line %d: EdgeBlocking runs EDGE_ONLY in the PUSH direction" % line)
            self.sched(label)
            push = self.edge_functor_for(args[0][1], "push", None, None)
            self.emit("gen::all_edges_blocked(c, G, %d, %s%s);" % (s1["blocking_size"], push, self.init_list(True)),
                      depth)
            self.notes.append("edges.apply at line %d: EdgeBlocking, destination segments of %d vertices"
                              % (line, s1["blocking_size"]))
        elif name == "apply" and target == ("id", self.prog.edges["name"]):
            sname = self.sched(label)
            push = self.edge_functor_for(args[0][1], "push", None, None)
            pull = self.edge_functor_for(args[0][1], "pull", None, None)
            self.needs_ids = True
            self.emit("if (%s.s1.direction == GG_PUSH) gen::all_edges_step(c, g, *ws, ids, %s.s1, %s%s);"
                      % (sname, sname, push, self.init_list(True)), depth)
            self.emit("else gen::all_edges_step(c, g, *ws, ids, %s.s1, %s%s);"
                      % (sname, pull, self.init_list(True)), depth)
        else:
            raise CompileError("line %d: unsupported call %s" % (line, name))


def generate(prog: Program, outputs: List[str]) -> (str, List[str]):
    """HIP C++ source of the module and the analysis notes."""
    for o in outputs:
        if o not in prog.vectors:
            raise CompileError("output %r is not a vector of the program" % o)
    notes: List[str] = []
    scheds = lower_schedules(prog)
    mg = MainGen(prog, scheds, notes)
    mg.stmts(prog.funcs["main"].body, 1)
    pre = []
    for s in prog.scalars:  # host scalars, in declaration order
        pre.append("    const double s_%s = (double)(%s);" % (s, mg.hexpr(prog.scalars[s]["init"])))
    for v, d in prog.vectors.items():
        ct = CTYPE[d["type"]]
        pre.append("    DevBuf<%s> vec_%s;" % (ct, v))
        pre.append("    vec_%s.ensure((size_t)g.n);" % v)
        init = d["init"]
        if init[0] == "method" and init[2] == "getOutDegrees":
            pre.append("    gen::out_degrees<%s>(c, g, vec_%s.p);" % (ct, v))
        else:
            pre.append("    gen::fill<%s>(c, vec_%s.p, g.n, (%s)(%s));" % (ct, v, ct, mg.hexpr(init)))
    cap = "(long long)g.n + g.m" if mg.no_dedup else "(long long)g.n"
    setup = ["    Ctx c;", "    c.s = reinterpret_cast<hipStream_t>(stream);", "    c.num_cus = G.num_cus;"]
    if mg.uses_edge_only:
        setup.append("    ensure_coo(c, G);")
    if mg.uses_pull:
        if prog.edges["weighted"]:
            # the transpose carries no weights: a weighted PULL reads in-edge weights in out-edge order
            setup.append("    require(G.symmetric, GG_ERR_UNSUPPORTED_SCHEDULE, "
                         "\"PULL over a weighted edgeset needs a symmetric graph\");")
        setup.append("    ensure_transpose(c, G);")
    setup += ["    Lease ws(G);", "    const DevGraph g = G.view();",
              "    auto arg = [&](int k) -> int64_t {",
              "        require(k < nargs, GG_ERR_INVALID_ARG, \"missing program argument\");",
              "        return args[k];", "    };"]
    fsetup = []
    if mg.frontiers:
        fsetup = ["    FrontierState fs(c, *ws, g.n, %s);" % cap,
                  "    ws->tags.ensure((size_t)g.n);", "    fill_i32(c, ws->tags.p, g.n, 0);",
                  "    int iter = 0;"]
    if mg.needs_ids:
        fsetup += ["    ws->aux_i32[0].ensure((size_t)g.n);",
                   "    hipLaunchKernelGGL(gen::k_gen_iota, dim3(blocks_for(g.n, kBlock, 8192)), dim3(kBlock), 0, "
                   "c.s, ws->aux_i32[0].p, g.n);",
                   "    GG_CHECK_LAUNCH();", "    const int32_t *ids = ws->aux_i32[0].p;"]
    copy = ["    require(outs != nullptr, GG_ERR_INVALID_ARG, \"output array is NULL\");"]
    for i, o in enumerate(outputs):
        copy.append("    require(outs[%d] != nullptr, GG_ERR_INVALID_ARG, \"output %s is NULL\");" % (i, o))
    for i, o in enumerate(outputs):
        ct = CTYPE[prog.vectors[o]["type"]]
        copy.append("    GG_HIP(hipMemcpyAsync(outs[%d], vec_%s.p, sizeof(%s) * (size_t)g.n, hipMemcpyDeviceToDevice, c.s));"
                    % (i, o, ct))
    copy.append("    GG_HIP(hipStreamSynchronize(c.s));")
    if prog.edges["weighted"]:
        setup.append("    require(G.has_weights, GG_ERR_INVALID_ARG, \"the program's edgeset is weighted\");")
    body = "\n".join(setup + pre + fsetup + mg.out + copy)
    src = """// Generated from a program in the algorithm and scheduling languages; do not edit.
#include "gen_rt.hpp"

using namespace gg;

namespace {
%s
}  // namespace

extern "C" gg_status gen_main(gg_graph *gh, const int64_t *args, int32_t nargs, void **outs, gg_stream_t stream) {
    try {
    require(gh != nullptr, GG_ERR_INVALID_ARG, "graph is NULL");
    Graph &G = gh->g;
%s
    g_last_error.clear();
    return GG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GG_ERR_DEVICE;
    }
}
""" % ("\n".join(list(mg.functors.values()) + mg.fused_kernels), body)
    return src, notes
