"""The GPU monitor's per-formula automata, restated step by step in Python and
checked against the oracle's three-valued semantics on random paths.

Each GPU monitor keeps O(1) registers per trajectory instead of the path
(Sec. 3.2 keeps a trace buffer).  The restatements below follow the device's
two hooks: `step` inspects a state just entered (index k, entry time t), and
`advance` sees the time tn at which that state is left (+inf: absorbing).
The first prefix at which an automaton decides, and its verdict, must equal
the first prefix the oracle's semantics decides.  This pins the reasoning
behind each automaton (which registers suffice); the HIP code itself is
compared with the oracle, trajectory by trajectory, by the GPU parity tests.
"""
import math

import numpy as np
import pytest

from oracle import bltlc
from test_oracle_semantics import _random_walk_trace, first_decided_point


def _run(st, tm, nt, step, advance):
    """Drive an automaton over a prefix; ((m, w), verdict) or (None, 2)."""
    for k in range(len(st)):
        v = step(k, tm[k], st[k])
        if v:
            return (k, 0), (1 if v == 1 else 0)
        tn = tm[k + 1] if k + 1 < len(st) else nt
        if tn is None:
            return None, 2
        v = advance(tn, math.isinf(tn))
        if v:
            return (k, 1), (1 if v == 1 else 0)
    return None, 2


def _flip(v, neg):
    return (3 - v if v else 0) if neg else v


def until(lo, hi, p1, p2, neg=False):
    """p1 U[lo,hi] p2 (negated for G): no registers."""
    def step(k, t, x):
        return _flip(1 if (lo <= t <= hi and p2(x)) else (2 if not p1(x) else 0), neg)

    def advance(tn, absorbing):
        return _flip(2 if (absorbing or tn > hi) else 0, neg)
    return step, advance


def response(lo, hi, d, p, q, neg=False):
    """G[lo,hi](p | F[0,d] q) (negated, with p, q negated, for F[lo,hi](p & G[0,d] q)):
    the entry time of the oldest open obligation."""
    r = {"tp": -1.0}

    def step(k, t, x):
        if lo <= t <= hi and not p(x) and r["tp"] < 0:
            r["tp"] = t
        if q(x):
            r["tp"] = -1.0
        return _flip(1 if (r["tp"] < 0 and t > hi) else 0, neg)

    def advance(tn, absorbing):
        if r["tp"] >= 0:
            return _flip(2 if (absorbing or tn - r["tp"] > d) else 0, neg)
        return _flip(1 if (absorbing or tn > hi) else 0, neg)
    return step, advance


def nested(lo, hi, c, p, q, s):
    """p U[lo,hi] (q U[0,c] s): whether p has held so far, the latest admissible start."""
    r = {"ok": True, "ts": -1.0}

    def step(k, t, x):
        if r["ok"] and lo <= t <= hi:
            r["ts"] = t
        hit = r["ts"] >= 0 and s(x)
        if not hit and not q(x):
            r["ts"] = -1.0
        r["ok"] = r["ok"] and p(x)
        return 1 if hit else (2 if (r["ts"] < 0 and (not r["ok"] or t > hi)) else 0)

    def advance(tn, absorbing):
        if r["ts"] >= 0 and (absorbing or tn - r["ts"] > c):
            r["ts"] = -1.0
        return 2 if (r["ts"] < 0 and (not r["ok"] or absorbing or tn > hi)) else 0
    return step, advance


def until_glob(lo, hi, c, p, q, s):
    """p U[lo,hi] (s & G[0,c] q): whether p has held so far, the earliest running start."""
    r = {"ok": True, "tc": -1.0}

    def step(k, t, x):
        if not q(x):
            r["tc"] = -1.0
        if r["tc"] < 0 and r["ok"] and lo <= t <= hi and q(x) and s(x):
            r["tc"] = t
        r["ok"] = r["ok"] and p(x)
        return 2 if (r["tc"] < 0 and (not r["ok"] or t > hi)) else 0

    def advance(tn, absorbing):
        if r["tc"] >= 0:
            return 1 if (absorbing or tn - r["tc"] > c) else 0
        return 2 if (not r["ok"] or absorbing or tn > hi) else 0
    return step, advance


def next_until(lo, hi, lo2, hi2, p, q, neg=False):
    """X[lo,hi](p U[lo2,hi2] q) (negated inside for G): the entry time of state 1."""
    r = {"t1": -1.0}

    def step(k, t, x):
        if k == 0:
            return 0
        if r["t1"] < 0:
            r["t1"] = t
        rel = t - r["t1"]
        return _flip(1 if (lo2 <= rel <= hi2 and q(x)) else (2 if not p(x) else 0), neg)

    def advance(tn, absorbing):
        if r["t1"] < 0:
            return 2 if (absorbing or not (lo <= tn <= hi)) else 0
        return _flip(2 if (absorbing or tn - r["t1"] > hi2) else 0, neg)
    return step, advance


def _cases(rng):
    a = float(rng.choice([0.0, rng.uniform(0, 2)]))
    b = a + float(rng.uniform(0.3, 5))
    c = float(rng.uniform(0.2, 2.5))
    a2 = float(rng.choice([0.0, rng.uniform(0, 1.5)]))
    b2 = a2 + float(rng.uniform(0.3, 4))
    i, j, m = (int(v) for v in rng.integers(0, 7, size=3))
    le = lambda n: (lambda x: x[0] <= n)   # noqa: E731
    ge = lambda n: (lambda x: x[0] >= n)   # noqa: E731
    notf = lambda f: (lambda x: not f(x))  # noqa: E731
    yield f"(X<={i}) U[{a!r},{b!r}] (X>={j})", until(a, b, le(i), ge(j))
    yield f"G[{a!r},{b!r}](X<={i})", until(a, b, lambda x: True, notf(le(i)), neg=True)
    yield f"G[{a!r},{b!r}](X<={i} | F[0,{c!r}](X>={j}))", response(a, b, c, le(i), ge(j))
    yield (f"F[{a!r},{b!r}]((X>={i}) & G[0,{c!r}](X<={j}))",
           response(a, b, c, notf(ge(i)), notf(le(j)), neg=True))
    yield (f"(X<={i}) U[{a!r},{b!r}] ((X>={j}) U[0,{c!r}] (X>={m}))",
           nested(a, b, c, le(i), ge(j), ge(m)))
    yield f"F[{a!r},{b!r}](F[0,{c!r}](X>={m}))", nested(a, b, c, lambda x: True, lambda x: True, ge(m))
    yield (f"(X<={i}) U[{a!r},{b!r}] ((X<={m}) & G[0,{c!r}](X>={j}))",
           until_glob(a, b, c, le(i), ge(j), le(m)))
    yield (f"X[0,{c!r}]((X<={i}) U[{a2!r},{b2!r}] (X>={j}))",
           next_until(0.0, c, a2, b2, le(i), ge(j)))
    yield (f"X[0,{c!r}](G[{a2!r},{b2!r}](X<={i}))",
           next_until(0.0, c, a2, b2, lambda x: True, notf(le(i)), neg=True))


@pytest.mark.parametrize("seed", range(4))
def test_automata_decide_where_the_semantics_decide(seed):
    rng = np.random.default_rng(100 + seed)
    seen = {0: 0, 1: 0, 2: 0}
    for _ in range(150):
        st, tm, nt = _random_walk_trace(rng, 14)
        if rng.random() < 0.3:
            nt = math.inf               # the last state is absorbing
        for text, (step, advance) in _cases(rng):
            exp_point, exp_v = first_decided_point(bltlc.parse(text, ["X"]), st, tm, nt)
            point, v = _run(st, tm, nt, step, advance)
            assert point == exp_point, (text, st.ravel().tolist(), tm.tolist(), nt)
            if point is not None:
                assert v == exp_v, (text, st.ravel().tolist(), tm.tolist(), nt)
            seen[v] += 1
    assert min(seen[0], seen[1]) > 100, seen     # both verdicts occur often
