"""BLTLc parser for the CPU oracle (test infrastructure only).

Grammar (Sec. 3.1, the BLTLc syntax):
    phi ::= val op val | !phi | phi & phi | phi | phi | X I phi | phi U I phi
            | F I phi | G I phi | (phi) | true | false
    val ::= name | number | val (+ - * /) val | -val | sqrt(val) | pow(val, val) | (val)
    I   ::= [a, b] | <= b | (omitted: [0, inf))
with op in {<, <=, >=, >, =, !=}.  Precedence: unary (!, X, F, G) binds
tightest, then U (right associative), then &, then |.

Finally and Globally are rewritten with the paper's equivalences (Sec. 3.1):
F^I p == (tt U^I p) and G^I p == not F^I not p.

The result is a flat node table consumed by oracle/smc_oracle.c.
"""
from __future__ import annotations

import math
import re
from dataclasses import dataclass, field

N_TRUE, N_FALSE, N_PRED, N_NOT, N_AND, N_OR, N_NEXT, N_UNTIL = range(8)
OPS = {"<": 0, "<=": 1, ">=": 2, ">": 3, "=": 4, "==": 4, "!=": 5}
E_VAR, E_CONST, E_ADD, E_SUB, E_MUL, E_DIV, E_NEG, E_SQRT, E_POW = range(9)

_TOKEN = re.compile(
    r"\s*(?:(?P<num>(?:\d+\.\d*|\.\d+|\d+)(?:[eE][+-]?\d+)?)|(?P<name>[A-Za-z_][A-Za-z_0-9]*)"
    r"|(?P<op><=|>=|!=|==|&&|\|\||[-+*/()<>=!&|\[\],]))"
)


class ParseError(ValueError):
    pass


def _tokenize(text):
    out, pos = [], 0
    text = text.strip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise ParseError(f"unexpected character at {pos}: {text[pos:pos + 10]!r}")
        pos = m.end()
        if m.group("num"):
            out.append(("num", m.group("num")))
        elif m.group("name"):
            out.append(("name", m.group("name")))
        else:
            tok = m.group("op")
            tok = {"&&": "&", "||": "|"}.get(tok, tok)
            out.append(("op", tok))
        while pos < len(text) and text[pos].isspace():
            pos += 1
    return out


@dataclass
class Formula:
    """Flat node table (post-order) plus predicate stack programs."""

    type: list = field(default_factory=list)
    a: list = field(default_factory=list)
    b: list = field(default_factory=list)
    lo: list = field(default_factory=list)
    hi: list = field(default_factory=list)
    pred: list = field(default_factory=list)
    pred_op: list = field(default_factory=list)
    lhs_off: list = field(default_factory=list)
    lhs_len: list = field(default_factory=list)
    rhs_off: list = field(default_factory=list)
    rhs_len: list = field(default_factory=list)
    prog_op: list = field(default_factory=list)
    prog_arg: list = field(default_factory=list)
    root: int = -1

    def node(self, t, a=-1, b=-1, lo=0.0, hi=math.inf, pred=-1):
        self.type.append(t)
        self.a.append(a)
        self.b.append(b)
        self.lo.append(float(lo))
        self.hi.append(float(hi))
        self.pred.append(pred)
        return len(self.type) - 1

    def predicate(self, lhs, op, rhs):
        self.pred_op.append(OPS[op])
        self.lhs_off.append(len(self.prog_op))
        for o, g in lhs:
            self.prog_op.append(o)
            self.prog_arg.append(float(g))
        self.lhs_len.append(len(lhs))
        self.rhs_off.append(len(self.prog_op))
        for o, g in rhs:
            self.prog_op.append(o)
            self.prog_arg.append(float(g))
        self.rhs_len.append(len(rhs))
        return len(self.pred_op) - 1

    @property
    def n_nodes(self):
        return len(self.type)


class _Parser:
    def __init__(self, text, names):
        self.toks = _tokenize(text)
        self.i = 0
        self.names = {n: k for k, n in enumerate(names)}
        self.f = Formula()

    # token helpers -----------------------------------------------------
    def peek(self, k=0):
        j = self.i + k
        return self.toks[j] if j < len(self.toks) else ("eof", "")

    def take(self):
        t = self.peek()
        self.i += 1
        return t

    def expect(self, val):
        t = self.take()
        if t[1] != val:
            raise ParseError(f"expected {val!r}, got {t[1]!r}")

    def is_op(self, val, k=0):
        t = self.peek(k)
        return t[0] == "op" and t[1] == val

    # formulas ----------------------------------------------------------
    def parse(self):
        root = self.disj()
        if self.peek()[0] != "eof":
            raise ParseError(f"trailing input at {self.peek()[1]!r}")
        self.f.root = root
        return self.f

    def disj(self):
        left = self.conj()
        while self.is_op("|"):
            self.take()
            right = self.conj()
            left = self.f.node(N_OR, left, right)
        return left

    def conj(self):
        left = self.until()
        while self.is_op("&"):
            self.take()
            right = self.until()
            left = self.f.node(N_AND, left, right)
        return left

    def until(self):
        left = self.unary()
        if self.peek() == ("name", "U"):
            self.take()
            lo, hi = self.interval()
            right = self.until()  # right associative
            return self.f.node(N_UNTIL, left, right, lo, hi)
        return left

    def interval(self):
        if self.is_op("["):
            self.take()
            lo = self.number()
            self.expect(",")
            hi = self.number()
            self.expect("]")
        elif self.is_op("<="):
            self.take()
            lo, hi = 0.0, self.number()
        else:
            lo, hi = 0.0, math.inf
        if not (0.0 <= lo <= hi):
            raise ParseError(f"bad interval [{lo}, {hi}]")
        return lo, hi

    def number(self):
        t = self.take()
        if t[0] == "name" and t[1] in ("inf", "Inf", "INF"):
            return math.inf
        if t[0] != "num":
            raise ParseError(f"expected a number, got {t[1]!r}")
        return float(t[1])

    def unary(self):
        t = self.peek()
        if t[0] == "op" and t[1] == "!":
            self.take()
            return self.f.node(N_NOT, self.unary())
        if t[0] == "name" and t[1] in ("F", "G", "X") and (
                t[1] not in self.names or self.is_op("[", 1)):
            # A species may share the letter of an operator; an interval right
            # after the letter always means the operator.
            self.take()
            lo, hi = self.interval()
            arg = self.unary()
            if t[1] == "X":
                return self.f.node(N_NEXT, arg, -1, lo, hi)
            tt = self.f.node(N_TRUE)
            if t[1] == "F":
                return self.f.node(N_UNTIL, tt, arg, lo, hi)
            neg = self.f.node(N_NOT, arg)
            fin = self.f.node(N_UNTIL, tt, neg, lo, hi)
            return self.f.node(N_NOT, fin)
        if t[0] == "name" and t[1] in ("true", "tt"):
            self.take()
            return self.f.node(N_TRUE)
        if t[0] == "name" and t[1] in ("false", "ff"):
            self.take()
            return self.f.node(N_FALSE)
        if self.is_op("("):
            # Either a parenthesised formula or a predicate starting with "(".
            save = self.i
            saved_len = (len(self.f.type), len(self.f.pred_op), len(self.f.prog_op))
            try:
                return self.predicate()
            except ParseError:
                self.i = save
                self._truncate(*saved_len)
            self.take()
            inner = self.disj()
            self.expect(")")
            return inner
        return self.predicate()

    def _truncate(self, n_nodes, n_preds, n_prog):
        f = self.f
        for lst in (f.type, f.a, f.b, f.lo, f.hi, f.pred):
            del lst[n_nodes:]
        for lst in (f.pred_op, f.lhs_off, f.lhs_len, f.rhs_off, f.rhs_len):
            del lst[n_preds:]
        del f.prog_op[n_prog:]
        del f.prog_arg[n_prog:]

    def predicate(self):
        lhs = self.val()
        t = self.take()
        if t[0] != "op" or t[1] not in OPS:
            raise ParseError(f"expected a comparison, got {t[1]!r}")
        rhs = self.val()
        k = self.f.predicate(lhs, t[1], rhs)
        return self.f.node(N_PRED, pred=k)

    # value expressions (stack programs) --------------------------------
    def val(self):
        prog = self.term()
        while self.is_op("+") or self.is_op("-"):
            op = self.take()[1]
            prog = prog + self.term() + [(E_ADD if op == "+" else E_SUB, 0)]
        return prog

    def term(self):
        prog = self.factor()
        while self.is_op("*") or self.is_op("/"):
            op = self.take()[1]
            prog = prog + self.factor() + [(E_MUL if op == "*" else E_DIV, 0)]
        return prog

    def factor(self):
        t = self.take()
        if t[0] == "num":
            return [(E_CONST, float(t[1]))]
        if t[0] == "op" and t[1] == "-":
            return self.factor() + [(E_NEG, 0)]
        if t[0] == "op" and t[1] == "(":
            p = self.val()
            self.expect(")")
            return p
        if t[0] == "name":
            low = t[1].lower()
            if low == "sqrt" and self.is_op("("):
                self.take()
                p = self.val()
                self.expect(")")
                return p + [(E_SQRT, 0)]
            if low == "pow" and self.is_op("("):
                self.take()
                p = self.val()
                self.expect(",")
                q = self.val()
                self.expect(")")
                return p + q + [(E_POW, 0)]
            if t[1] in self.names:
                return [(E_VAR, self.names[t[1]])]
            raise ParseError(f"unknown species {t[1]!r}")
        raise ParseError(f"unexpected token {t[1]!r}")


def parse(text: str, names) -> Formula:
    """Parse BLTLc text over the given species names into a node table."""
    return _Parser(text, list(names)).parse()
