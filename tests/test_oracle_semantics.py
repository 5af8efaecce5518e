"""Pins for the oracle's BLTLc semantics and its on-the-fly stopping point.

- golden traces whose verdicts and decision points were derived by hand from
  the semantics (Sec. 3.1) and the stop-at-first-decision rule (Sec. 3.2);
- the bisection search of the C driver against a brute-force scan of every
  prefix of real SSA paths;
- the verdict at the stopping point against the verdict on a path long enough
  to cover the whole time horizon;
- the F / G duality G p == not F not p (Sec. 3.1).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bltlc
from paper_0912_2551_amd import workloads as W

REASONS = {"state": oracle.R_STATE, "time": oracle.R_TIME, "absorbing": oracle.R_ABSORB}


def first_decided_point(f, states, times, next_time):
    """Brute force: evaluate every prefix in order, return ((m, w), value)."""
    n = len(states)
    for m in range(n):
        v = oracle.eval_prefix(f, states[: m + 1], times[: m + 1], None)
        if v != 2:
            return (m, 0), v
        nt = times[m + 1] if m + 1 < n else next_time
        if nt is None:
            continue
        v = oracle.eval_prefix(f, states[: m + 1], times[: m + 1], nt)
        if v != 2:
            return (m, 1), v
    return None, 2


def _golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "semantics_traces.json")) as fh:
        data = json.load(fh)
    for tr in data["traces"]:
        for case in tr["cases"]:
            yield pytest.param(tr, case, id=f"{tr['name']}:{case['formula']}")


@pytest.mark.parametrize("trace,case", list(_golden()))
def test_golden_trace(trace, case):
    f = bltlc.parse(case["formula"], trace["names"])
    states = np.asarray(trace["states"], dtype=np.int32)
    times = np.asarray(trace["times"], dtype=np.float64)
    nt = trace["next_time"]
    nt = math.inf if nt == "inf" else nt
    point, v = first_decided_point(f, states, times, nt)
    assert point == tuple(case["point"]), case["why"]
    assert v == case["verdict"], case["why"]
    m, w = point
    reason = "state" if w == 0 else ("absorbing" if (m + 1 >= len(times) and math.isinf(nt)) else "time")
    assert reason == case["reason"]


def test_parser_precedence():
    # U binds tighter than &, & tighter than |; F/G are rewritten per Sec. 3.1.
    f = bltlc.parse("(P<500) U[0,60] (S<=200) & G[0,60](E>=10)", ["E", "S", "ES", "P"])
    assert f.type[f.root] == bltlc.N_AND
    left = f.a[f.root]
    right = f.b[f.root]
    assert f.type[left] == bltlc.N_UNTIL and f.hi[left] == 60.0
    assert f.type[right] == bltlc.N_NOT                     # G = not F not
    fin = f.a[right]
    assert f.type[fin] == bltlc.N_UNTIL and f.type[f.a[fin]] == bltlc.N_TRUE
    assert f.type[f.b[fin]] == bltlc.N_NOT
    g = bltlc.parse("a>1 | b>1 & a>0 U b>2", ["a", "b"])
    assert g.type[g.root] == bltlc.N_OR
    with pytest.raises(bltlc.ParseError):
        bltlc.parse("F[0,1](Y>1)", ["X"])
    with pytest.raises(bltlc.ParseError):
        bltlc.parse("F[2,1](X>1)", ["X"])


def _random_walk_trace(rng, n, S=1):
    states = np.cumsum(rng.integers(-1, 2, size=(n, S)), axis=0).astype(np.int32) + 3
    times = np.concatenate([[0.0], np.cumsum(rng.exponential(0.5, size=n))])
    return states, times[:n], float(times[n])


DUALITY = [
    ("G[0,{T}](X>={c})", "!F[0,{T}](X<{c})"),
    ("G[{a},{T}](X<={c})", "!F[{a},{T}](!(X<={c}))"),
    ("F[0,{T}](X>={c})", "true U[0,{T}] (X>={c})"),
    # response and its dual, the identity the GPU monitor compiler relies on
    ("F[{a},{T}]((X>={c}) & G[0,1](X<=5))", "!G[{a},{T}](!(X>={c}) | F[0,1](!(X<=5)))"),
]


@pytest.mark.parametrize("lhs,rhs", DUALITY)
def test_duality_on_random_traces(lhs, rhs):
    rng = np.random.default_rng(7)
    for _ in range(200):
        st, tm, nt = _random_walk_trace(rng, 12)
        T = float(rng.uniform(0.5, 6))
        a = float(rng.uniform(0, 0.5)) * T
        c = int(rng.integers(0, 7))
        fa = bltlc.parse(lhs.format(T=T, a=a, c=c), ["X"])
        fb = bltlc.parse(rhs.format(T=T, a=a, c=c), ["X"])
        for m in range(len(st)):
            for nxt in (None, tm[m + 1] if m + 1 < len(tm) else nt):
                assert oracle.eval_prefix(fa, st[: m + 1], tm[: m + 1], nxt) == \
                    oracle.eval_prefix(fb, st[: m + 1], tm[: m + 1], nxt)


def _response_on_path(st, tm, lo, hi, d, p, q):
    """G[lo,hi](p | F[0,d] q) on a complete path whose last state is
    absorbing, straight from the definition: every position entered in
    [lo, hi] satisfies p, or some position at or after it, entered at most d
    later, satisfies q."""
    n = len(st)
    for i in range(n):
        if lo <= tm[i] <= hi and not p(st[i]):
            if not any(q(st[j]) and tm[j] - tm[i] <= d for j in range(i, n)):
                return 0
    return 1


def _persistence_on_path(st, tm, lo, hi, d, p, q):
    """F[lo,hi](p & G[0,d] q) on a complete path, from the definition: some
    position entered in [lo, hi] satisfies p, and q holds at it and at every
    later position entered at most d after it."""
    n = len(st)
    for i in range(n):
        if lo <= tm[i] <= hi and p(st[i]):
            if all(q(st[j]) for j in range(i, n) if tm[j] - tm[i] <= d):
                return 1
    return 0


def test_response_forms_on_complete_paths():
    """The oracle's nested evaluation of G I (p | F[0,d] q) and F I (p & G[0,d] q)
    against the definitions above, on random absorbing paths; both values
    occur often."""
    rng = np.random.default_rng(5)
    seen = {0: 0, 1: 0}
    for _ in range(300):
        st, tm, _ = _random_walk_trace(rng, 14)
        lo = float(rng.choice([0.0, rng.uniform(0, 2)]))
        hi = lo + float(rng.uniform(0.5, 6))
        d = float(rng.uniform(0.2, 2.5))
        c1, c2 = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        fr = bltlc.parse(f"G[{lo!r},{hi!r}](X<={c1} | F[0,{d!r}](X>={c2}))", ["X"])
        fp = bltlc.parse(f"F[{lo!r},{hi!r}]((X>={c1}) & G[0,{d!r}](X<={c2}))", ["X"])
        vr = oracle.eval_prefix(fr, st, tm, math.inf)
        vp = oracle.eval_prefix(fp, st, tm, math.inf)
        assert vr == _response_on_path(st, tm, lo, hi, d, lambda x: x[0] <= c1, lambda x: x[0] >= c2)
        assert vp == _persistence_on_path(st, tm, lo, hi, d, lambda x: x[0] >= c1, lambda x: x[0] <= c2)
        seen[vr] += 1
        seen[vp] += 1
    assert min(seen.values()) > 100, seen


def test_kleene_monotone_on_prefixes():
    """Once a prefix decides the formula, every longer prefix gives the same value."""
    rng = np.random.default_rng(11)
    f = bltlc.parse("(X<=6) U[0,4] ((X>=2) U[0,1.5] (X>=5)) | G[0,3](X>=1)", ["X"])
    for _ in range(100):
        st, tm, nt = _random_walk_trace(rng, 15)
        seen = None
        for m in range(len(st)):
            for nxt in (None, tm[m + 1] if m + 1 < len(tm) else nt):
                v = oracle.eval_prefix(f, st[: m + 1], tm[: m + 1], nxt)
                if seen is not None:
                    assert v == seen
                elif v != 2:
                    seen = v


def death_only():
    """X -> 0 at rate X from 30: absorbed at X = 0 after 30 events."""
    return W.from_reactions(["X"], [30], [(["X"], [], 1.0)], "death")


CASES = [
    (W.immigration_death, "F[0,10](X>=12)", 0),
    (W.immigration_death, "G[0,5](X<=30) & F[0,8](X>=40)", 0),
    (W.immigration_death, "(X<=60) U[0,20] ((X>=20) U[0,3] (X>=70))", 0),
    (W.isomerization, "(B<=30) U[0,3] (A<=20)", 0),
    (W.isomerization, "X[0,0.05](B>=1) | F[1,2](A<=15)", 0),
    (W.michaelis_menten, W.C2_FORMULA, 0),
    (W.michaelis_menten, "F[0,0.2](ES>=60)", 0),
    (W.dimerization, "F[0,5](A<=10)", 0),
    (W.immigration_death, "F[0,100](X>=120)", 50),   # event cap
    (death_only, "F[0,100](X>=40)", 0),               # decided only by absorption: FALSE
    (death_only, "G[0,100](X>=0)", 0),                # decided only by absorption: TRUE
]


@pytest.mark.parametrize("make,text,cap", CASES)
def test_driver_matches_brute_force(make, text, cap):
    """The bisection in the C driver finds the same first decided prefix as a
    scan over all prefixes of the same SSA path."""
    net = make()
    f = oracle.parse(text, net)
    ev, vd, rs = oracle.trajectories(net, f, 0, 24, seed=3, max_events=cap)
    for i in range(24):
        n_steps = int(ev[i]) + 2
        states, times, a0, absorbed = oracle.path(net, i, n_steps, seed=3)
        nt = math.inf if absorbed else None
        if cap:
            states, times = states[: cap + 1], times[: cap + 1]
        point, v = first_decided_point(f, states, times, nt)
        if point is None:
            assert cap and ev[i] == cap and vd[i] == 0 and rs[i] == oracle.R_CAP
            continue
        assert point[0] == ev[i], (i, point, ev[i])
        assert v == vd[i]
        m, w = point
        exp_reason = oracle.R_STATE if w == 0 else (oracle.R_ABSORB if (absorbed and m == len(states) - 1) else oracle.R_TIME)
        assert rs[i] == exp_reason


def test_verdict_matches_full_horizon_path():
    """The early verdict equals the verdict on a path covering the horizon."""
    net = W.immigration_death()
    f = oracle.parse("F[0,20](X>=25) & G[0,20](X<=60)", net)
    ev, vd, rs = oracle.trajectories(net, f, 0, 64, seed=9)
    for i in range(64):
        states, times, _, absorbed = oracle.path(net, i, 2000, seed=9)
        assert times[-1] > 20.0
        v = oracle.eval_prefix(f, states, times, None)
        assert v == vd[i]


def test_tmax_pessimistic_rule_and_cap():
    """Sec. 3.2: an unbounded formula undecided at t_max is FALSE; the event
    cap gives FALSE with the cap reason."""
    net = W.immigration_death()
    f = oracle.parse("F(X>=1000)", net)
    ev, vd, rs = oracle.trajectories(net, f, 0, 16, t_max=5.0)
    assert (vd == 0).all() and (rs == oracle.R_TMAX).all()
    for i in range(16):
        states, times, _, _ = oracle.path(net, i, int(ev[i]) + 1)
        assert times[ev[i]] <= 5.0 < times[ev[i] + 1]
    f2 = oracle.parse(W.C1_FORMULA, net)
    ev, vd, rs = oracle.trajectories(net, f2, 0, 16, max_events=10)
    assert (ev == 10).all() and (vd == 0).all() and (rs == oracle.R_CAP).all()


def _random_formula(rng, depth):
    """A random BLTLc formula over X and Y: predicates, boolean operators,
    next and until with windows that may start above 0, nested to `depth`."""
    if depth == 0 or rng.random() < 0.25:
        sp = "XY"[int(rng.integers(0, 2))]
        return f"{sp}{['<=', '>=', '<', '>'][int(rng.integers(0, 4))]}{int(rng.integers(0, 7))}"
    lo = float(rng.choice([0.0, rng.uniform(0, 1.5)]))
    hi = lo + float(rng.uniform(0.2, 4.0))
    k = int(rng.integers(0, 8))
    a = _random_formula(rng, depth - 1)
    if k == 0:
        return f"!({a})"
    if k == 1:
        return f"({a}) & ({_random_formula(rng, depth - 1)})"
    if k == 2:
        return f"({a}) | ({_random_formula(rng, depth - 1)})"
    if k == 3:
        return f"X[{lo!r},{hi!r}]({a})"
    if k == 4:
        return f"F[{lo!r},{hi!r}]({a})"
    if k == 5:
        return f"G[{lo!r},{hi!r}]({a})"
    return f"({a}) U[{lo!r},{hi!r}] ({_random_formula(rng, depth - 1)})"


def test_skip_scan_equals_plain_scan():
    """The until evaluation that jumps over positions where the left operand
    holds and the right one fails gives the same three-valued value as the
    scan over every position (the definition as written), on every prefix of
    random paths under random nested formulas, and the same stopping points
    on SSA paths."""
    rng = np.random.default_rng(23)
    decided = 0
    try:
        for _ in range(400):
            text = _random_formula(rng, 3)
            f = bltlc.parse(text, ["X", "Y"])
            st, tm, nt = _random_walk_trace(rng, 18, S=2)
            for m in range(0, len(st), 3):
                for nxt in (None, tm[m + 1] if m + 1 < len(tm) else nt, math.inf):
                    oracle.set_plain_scan(False)
                    fast = oracle.eval_prefix(f, st[: m + 1], tm[: m + 1], nxt)
                    oracle.set_plain_scan(True)
                    plain = oracle.eval_prefix(f, st[: m + 1], tm[: m + 1], nxt)
                    assert fast == plain, (text, m, nxt)
                    decided += fast != 2
        net = W.c3_network()
        for text in (W.nested_until_formula(net, 2), W.nested_until_formula(net, 5)):
            oracle.set_plain_scan(True)
            plain = oracle.trajectories(net, text, 0, 48, seed=1)
            oracle.set_plain_scan(False)
            fast = oracle.trajectories(net, text, 0, 48, seed=1)
            for a, b in zip(plain, fast):
                assert np.array_equal(a, b)
    finally:
        oracle.set_plain_scan(False)
    assert decided > 1000
