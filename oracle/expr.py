"""User element functions written as arithmetic expressions in x (agents of type FUNCTION,
Section 3.2; the paper compiles such agents into the generated kernel, Section 5).

Grammar (whitespace ignored):
    expr    := term (("+" | "-") term)*
    term    := unary (("*" | "/") unary)*
    unary   := "-" unary | primary
    primary := number | "x" | "(" expr ")" | ("sqrt" | "abs" | "exp") "(" expr ")"
    number  := decimal literal (digits, optional fraction, optional exponent)

Value: every literal is rounded to binary32 when the function is composed; every operation
(+, -, *, /, unary minus, sqrt, abs, exp) gives the correctly rounded binary32 result of its
exact value on binary32 operands, evaluated in the order the grammar gives (left to right
within a precedence level).  exp is the correctly rounded exp of the library's other agents.
"""
from __future__ import annotations

import re

import numpy as np

from .elem import exp_rn32

_TOKEN = re.compile(r"\s*(?:(\d+\.?\d*(?:[eE][+-]?\d+)?|\.\d+(?:[eE][+-]?\d+)?)|([A-Za-z_]+)|(.))")


def tokenize(s: str) -> list:
    out, pos = [], 0
    s = s.rstrip()
    while pos < len(s):
        m = _TOKEN.match(s, pos)
        if not m or m.end() == pos:
            raise ValueError(f"bad character at {pos} in {s!r}")
        num, name, ch = m.groups()
        pos = m.end()
        if num is not None:
            out.append(("num", float(num)))
        elif name is not None:
            out.append(("name", name))
        elif ch is not None and ch.strip():
            out.append(("op", ch))
    return out


class _Parser:
    def __init__(self, s: str):
        self.toks = tokenize(s)
        self.i = 0

    def peek(self):
        return self.toks[self.i] if self.i < len(self.toks) else ("end", None)

    def take(self, kind, val=None):
        t = self.peek()
        if t[0] != kind or (val is not None and t[1] != val):
            raise ValueError(f"expected {val or kind}, found {t[1]!r}")
        self.i += 1
        return t

    def expr(self):
        node = self.term()
        while self.peek() in (("op", "+"), ("op", "-")):
            op = self.take("op")[1]
            node = (op, node, self.term())
        return node

    def term(self):
        node = self.unary()
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take("op")[1]
            node = (op, node, self.unary())
        return node

    def unary(self):
        if self.peek() == ("op", "-"):
            self.take("op", "-")
            return ("neg", self.unary())
        return self.primary()

    def primary(self):
        t = self.peek()
        if t[0] == "num":
            self.i += 1
            return ("const", float(np.float32(t[1])))  # rounded to binary32 at composition
        if t == ("name", "x"):
            self.i += 1
            return ("x",)
        if t[0] == "name" and t[1] in ("sqrt", "abs", "exp"):
            self.i += 1
            self.take("op", "(")
            arg = self.expr()
            self.take("op", ")")
            return (t[1], arg)
        if t == ("op", "("):
            self.i += 1
            node = self.expr()
            self.take("op", ")")
            return node
        raise ValueError(f"unexpected {t[1]!r}")


def parse(s: str):
    p = _Parser(s)
    tree = p.expr()
    if p.peek()[0] != "end":
        raise ValueError(f"unexpected {p.peek()[1]!r} after the expression")
    return tree


def _rn(v):
    with np.errstate(all="ignore"):
        return np.asarray(v, dtype=np.float64).astype(np.float32)


def evaluate(tree, x: np.ndarray) -> np.ndarray:
    """Value of the expression tree on every binary32 element of x."""
    x = np.asarray(x, np.float32)
    kind = tree[0]
    if kind == "x":
        return x.copy()
    if kind == "const":
        return np.full(x.shape, tree[1], np.float32)
    if kind == "neg":
        return (-evaluate(tree[1], x)).astype(np.float32)
    if kind == "abs":
        return np.abs(evaluate(tree[1], x))
    if kind == "sqrt":
        with np.errstate(invalid="ignore"):
            return _rn(np.sqrt(evaluate(tree[1], x).astype(np.float64)))
    if kind == "exp":
        return exp_rn32(evaluate(tree[1], x))
    a = evaluate(tree[1], x).astype(np.float64)
    b = evaluate(tree[2], x).astype(np.float64)
    with np.errstate(all="ignore"):
        # + - * / of binary32 values: the float64 result rounded once is correctly rounded
        return _rn({"+": a + b, "-": a - b, "*": a * b, "/": a / b}[kind])


def apply_expr(src: str, x: np.ndarray) -> np.ndarray:
    return evaluate(parse(src), x)
