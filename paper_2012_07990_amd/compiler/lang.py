"""Lexer and parser for the subset of the algorithm and scheduling languages
(Algorithm Language and Scheduling Language sections) that the compiler
lowers: element and constant declarations, edge / vertex / filter functions,
a main function with frontier loops, counted loops and operator calls, and a
`schedule:` section of SimpleGPUSchedule / HybridGPUSchedule statements.

The parser builds plain tuples; `Program` keeps the declarations by kind.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple


class CompileError(ValueError):
    pass


_TOKEN = re.compile(r"""
    (?P<ws>[ \t\r\n]+|%[^\n]*|//[^\n]*)
  | (?P<label>\#[A-Za-z_][A-Za-z_0-9]*\#)
  | (?P<str>"[^"\n]*")
  | (?P<num>\d+\.\d*(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)
  | (?P<minassign>min=)
  | (?P<id>[A-Za-z_][A-Za-z_0-9]*)
  | (?P<op>->|==|!=|<=|>=|\+=|&&|\|\||[-+*/<>=!:;,(){}\[\].])
""", re.VERBOSE)


def tokenize(src: str) -> List[Tuple[str, str, int]]:
    out, pos, line = [], 0, 1
    while pos < len(src):
        m = _TOKEN.match(src, pos)
        if not m:
            raise CompileError("line %d: unexpected character %r" % (line, src[pos]))
        kind = m.lastgroup
        text = m.group(kind)
        if kind != "ws":
            out.append((kind, text, line))
        line += text.count("\n")
        pos = m.end()
    out.append(("eof", "", line))
    return out


@dataclass
class Func:
    name: str
    params: List[Tuple[str, str]]   # (name, type)
    result: Optional[Tuple[str, str]]  # (name, type) for `-> output : bool`
    body: list


@dataclass
class Program:
    elements: List[str] = field(default_factory=list)
    edges: Optional[dict] = None                     # {"name", "weighted"}
    vertices: Optional[str] = None                   # the vertexset name
    vectors: Dict[str, dict] = field(default_factory=dict)   # name -> {"type", "init"}
    scalars: Dict[str, dict] = field(default_factory=dict)   # name -> {"type", "init"}
    funcs: Dict[str, Func] = field(default_factory=dict)
    pqs: Dict[str, dict] = field(default_factory=dict)   # priority queues: name -> {"type"}
    schedule: list = field(default_factory=list)     # scheduling statements (tuples)


class Parser:
    def __init__(self, src: str):
        self.toks = tokenize(src)
        self.i = 0

    # -- token helpers ----------------------------------------------------------
    def peek(self, k=0):
        return self.toks[min(self.i + k, len(self.toks) - 1)]

    def next(self):
        t = self.toks[self.i]
        self.i += 1
        return t

    def at(self, text):
        return self.peek()[1] == text and self.peek()[0] != "eof"

    def expect(self, text):
        t = self.next()
        if t[1] != text:
            raise CompileError("line %d: expected %r, found %r" % (t[2], text, t[1]))
        return t

    def ident(self):
        t = self.next()
        if t[0] != "id":
            raise CompileError("line %d: expected a name, found %r" % (t[2], t[1]))
        return t[1]

    # -- types -----------------------------------------------------------------------
    def type_(self):
        name = self.ident()
        if name == "edgeset":
            self.expect("{"); self.ident(); self.expect("}")
            self.expect("(")
            parts = [self.ident()]
            while self.at(","):
                self.next()
                parts.append(self.ident())
            self.expect(")")
            return ("edgeset", len(parts) == 3)
        if name == "vertexset":
            self.expect("{"); self.ident(); self.expect("}")
            return ("vertexset",)
        if name == "vector":
            self.expect("{"); self.ident(); self.expect("}")
            self.expect("(")
            elem = self.ident()
            self.expect(")")
            return ("vector", elem)
        if name == "priority_queue":
            self.expect("{"); self.ident(); self.expect("}")
            self.expect("(")
            elem = self.ident()
            self.expect(")")
            return ("pq", elem)
        return ("scalar", name)

    # -- expressions ------------------------------------------------------------------
    def expr(self):
        return self.binary(0)

    _PREC = [("||",), ("&&",), ("==", "!="), ("<", ">", "<=", ">="), ("+", "-"), ("*", "/")]

    def binary(self, level):
        if level == len(self._PREC):
            return self.unary()
        lhs = self.binary(level + 1)
        while self.peek()[0] == "op" and self.peek()[1] in self._PREC[level]:
            op = self.next()[1]
            rhs = self.binary(level + 1)
            lhs = ("bin", op, lhs, rhs)
        return lhs

    def unary(self):
        if self.at("-") or self.at("!"):
            op = self.next()[1]
            return ("un", op, self.unary())
        return self.postfix(self.primary())

    def primary(self):
        t = self.next()
        if t[0] == "num":
            return ("num", t[1])
        if t[1] == "(":
            e = self.expr()
            self.expect(")")
            return e
        if t[1] == "new":
            ty = self.type_()
            return ("new", ty, self.args())
        if t[0] == "id":
            if t[1] in ("true", "false"):
                return ("bool", t[1] == "true")
            return ("id", t[1])
        raise CompileError("line %d: unexpected %r" % (t[2], t[1]))

    def args(self):
        self.expect("(")
        out = []
        if not self.at(")"):
            out.append(self.expr())
            while self.at(","):
                self.next()
                out.append(self.expr())
        self.expect(")")
        return out

    def postfix(self, e):
        while True:
            if self.at("["):
                self.next()
                idx = self.expr()
                self.expect("]")
                e = ("index", e, idx)
            elif self.at("."):
                self.next()
                name = self.ident()
                e = ("method", e, name, self.args() if self.at("(") else [])
            elif self.at("(") and e[0] == "id":
                e = ("call", e[1], self.args())
            else:
                return e

    # -- statements -----------------------------------------------------------------------
    def block(self, *ends):
        out = []
        while not any(self.at(x) for x in ends):
            if self.peek()[0] == "eof":
                raise CompileError("unexpected end of input (missing %s)" % "/".join(ends))
            out.append(self.statement())
        return out

    def statement(self):
        label = None
        if self.peek()[0] == "label":
            label = self.next()[1].strip("#")
        line = self.peek()[2]
        if self.at("var"):
            self.next()
            name = self.ident()
            self.expect(":")
            ty = self.type_()
            init = None
            if self.at("="):
                self.next()
                init = self.expr()
            self.expect(";")
            return ("var", name, ty, init, label, line)
        if self.at("while"):
            self.next()
            self.expect("(")
            cond = self.expr()
            self.expect(")")
            body = self.block("end")
            self.expect("end")
            return ("while", cond, body, label, line)
        if self.at("for"):
            self.next()
            var = self.ident()
            self.expect("in")
            lo = self.expr()
            self.expect(":")
            hi = self.expr()
            body = self.block("end")
            self.expect("end")
            return ("for", var, lo, hi, body, label, line)
        if self.at("delete"):
            self.next()
            name = self.ident()
            self.expect(";")
            return ("delete", name, label, line)
        lhs = self.expr()
        if self.peek()[0] == "minassign" or self.at("=") or self.at("+="):
            op = self.next()[1]
            rhs = self.expr()
            self.expect(";")
            return ("assign", op, lhs, rhs, label, line)
        self.expect(";")
        return ("expr", lhs, label, line)

    # -- declarations -------------------------------------------------------------------------
    def program(self) -> Program:
        p = Program()
        while self.peek()[0] != "eof":
            if self.at("element"):
                self.next()
                p.elements.append(self.ident())
                self.expect("end")
            elif self.at("const"):
                self.next()
                name = self.ident()
                self.expect(":")
                ty = self.type_()
                init = None
                if ty[0] == "pq":
                    if self.at("="):
                        raise CompileError("line %d: a priority queue is created in main "
                                           "(pq = new priority_queue{Vertex}(int)(vector, start))" % self.peek()[2])
                else:
                    self.expect("=")
                    init = self.expr()
                self.expect(";")
                if ty[0] == "pq":
                    p.pqs[name] = {"type": ty[1]}
                elif ty[0] == "edgeset":
                    p.edges = {"name": name, "weighted": ty[1]}
                elif ty[0] == "vertexset":
                    p.vertices = name
                elif ty[0] == "vector":
                    p.vectors[name] = {"type": ty[1], "init": init}
                else:
                    p.scalars[name] = {"type": ty[1], "init": init}
            elif self.at("func"):
                self.next()
                name = self.ident()
                self.expect("(")
                params = []
                while not self.at(")"):
                    pn = self.ident()
                    self.expect(":")
                    params.append((pn, self.ident()))
                    if self.at(","):
                        self.next()
                self.expect(")")
                result = None
                if self.at("->"):
                    self.next()
                    rn = self.ident()
                    self.expect(":")
                    result = (rn, self.ident())
                body = self.block("end")
                self.expect("end")
                p.funcs[name] = Func(name, params, result, body)
            elif self.at("schedule"):
                self.next()
                self.expect(":")
                p.schedule = self.block_until_eof()
            else:
                t = self.peek()
                raise CompileError("line %d: unexpected %r at top level" % (t[2], t[1]))
        if p.edges is None:
            raise CompileError("the program declares no edgeset")
        if "main" not in p.funcs:
            raise CompileError("the program has no main function")
        return p

    def block_until_eof(self):
        """The scheduling language: schedule objects, their config calls and
        program->applyGPUSchedule("label", object). Returns tuples
        ("decl", kind, name, args) / ("config", name, method, args) /
        ("apply", label, name)."""
        out = []

        def sargs():
            self.expect("(")
            vals = []
            while not self.at(")"):
                t = self.next()
                if t[0] == "str":
                    vals.append(("str", t[1][1:-1]))
                elif t[0] == "num":
                    vals.append(("num", t[1]))
                elif t[0] == "id":
                    vals.append(("id", t[1]))
                else:
                    raise CompileError("line %d: unexpected %r in a schedule call" % (t[2], t[1]))
                if self.at(","):
                    self.next()
            self.expect(")")
            return vals

        while self.peek()[0] != "eof":
            t = self.next()
            if t[1] in ("SimpleGPUSchedule", "HybridGPUSchedule"):
                name = self.ident()
                args = sargs() if self.at("(") else []
                self.expect(";")
                out.append(("decl", t[1], name, args))
            elif t[1] == "program":
                self.expect("->")
                method = self.ident()
                args = sargs()
                self.expect(";")
                if method != "applyGPUSchedule" or len(args) != 2 or args[0][0] != "str":
                    raise CompileError("line %d: expected program->applyGPUSchedule(\"label\", schedule)" % t[2])
                out.append(("apply", args[0][1], args[1][1]))
            elif t[0] == "id":
                self.expect(".")
                method = self.ident()
                args = sargs()
                self.expect(";")
                out.append(("config", t[1], method, args))
            else:
                raise CompileError("line %d: unexpected %r in the schedule" % (t[2], t[1]))
        return out


def parse(src: str) -> Program:
    return Parser(src).program()
