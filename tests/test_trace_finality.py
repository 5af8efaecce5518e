"""The final-position rule of incremental trace-program evaluation, checked
against the oracle's three-valued semantics of prefixes (Sec. 3.1, 3.2),
without the GPU.

The GPU evaluates a formula outside the compact monitor classes on the
recorded prefix of a trajectory, incrementally: after a test that leaves the
formula open, each node of the formula keeps the count of its leading
positions whose values no longer prefix can change, and later tests
recompute only the positions from that count on.  The rule, per node,
children first, for a prefix of m states (the time the last one is left not
yet known):
  - true, false, a predicate: position i < m;
  - NOT, AND, OR: the operands are final at i;
  - NEXT: i + 1 < m and the operand is final at i + 1;
  - UNTIL over [lo, hi], hi finite: some position j < m, below both operands'
    final counts, is entered more than hi after state i.  Entry times do not
    decrease, so these i form a prefix of the positions.
The pins: on real trajectories of three models, for formulas of every
operator and nesting used by the GPU parity cases and for 40 random nested
formulas, and at many prefix lengths, every position the rule calls final has a known value (T or F) on
the prefix, and the same value on longer prefixes and on the whole
trajectory.  Planted mistakes in the rule (NEXT one position too far, an
until that ignores its operands' finality, one that counts the position just
inside its window) each claim a position whose value still changes.
"""
import ctypes
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle import bltlc
from paper_0912_2551_amd import workloads as W

from formula_gen import random_formula

U = 2   # the oracle's "unknown"


def final_counts(f, times, m, mutant=None):
    """Final-position count of every node of f for the prefix of m states."""
    F = [0] * f.n_nodes
    for q in range(f.n_nodes):   # post-order: operands come first
        t, a, b = f.type[q], f.a[q], f.b[q]
        if t in (bltlc.N_TRUE, bltlc.N_FALSE, bltlc.N_PRED):
            F[q] = m
        elif t == bltlc.N_NOT:
            F[q] = F[a]
        elif t in (bltlc.N_AND, bltlc.N_OR):
            F[q] = min(F[a], F[b])
        elif t == bltlc.N_NEXT:
            F[q] = min(m, F[a]) if mutant == "next" else max(0, min(m - 1, F[a] - 1))
        elif t == bltlc.N_UNTIL:
            hi = f.hi[q]
            if math.isinf(hi):
                F[q] = 0
                continue
            fp = m - 1 if mutant == "until-operands" else min(F[a], F[b], m - 1)
            if fp <= 0:
                F[q] = 0
                continue
            past = (lambda i: times[fp] - times[i] >= hi) if mutant == "until-window" else \
                (lambda i: times[fp] - times[i] > hi)
            i = 0
            while i <= fp and past(i):
                i += 1
            F[q] = i
    return F


class Values:
    """Value of node q at position i on the prefix of m states (the oracle's
    evaluation of the subformula rooted at q, on the states from i on: the
    semantics only see entry-time differences), with each subformula's
    tables built once."""

    def __init__(self, f, states, times):
        self.st = np.ascontiguousarray(states, dtype=np.int32).reshape(len(states), -1)
        self.t = np.asarray(times, dtype=np.float64)
        self.forms = [oracle._Form(dataclasses.replace(f, root=q)) for q in range(f.n_nodes)]

    def __call__(self, q, i, m, next_time=None):
        st = np.ascontiguousarray(self.st[i:m])
        t = np.zeros(m - i + 1, dtype=np.float64)
        t[:m - i] = self.t[i:m]
        if next_time is not None:
            t[m - i] = next_time
        return oracle.lib().oracle_eval(ctypes.c_int32(st.shape[1]), *self.forms[q].args(), ctypes.c_int64(m - i),
                                        ctypes.c_int32(0 if next_time is None else 1),
                                        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def violations(f, states, times, absorbed, prefixes, mutant=None, per_node=40, rng=None):
    """Positions the rule calls final whose value is unknown on the prefix or
    differs on a longer prefix or on the whole trajectory."""
    n = len(states)
    full_next = math.inf if absorbed else None
    value = Values(f, states, times)
    bad = []
    for m in prefixes:
        if m > n:
            continue
        F = final_counts(f, times, m, mutant)
        for q in range(f.n_nodes):
            if F[q] == 0:
                continue
            pos = np.arange(F[q])
            if len(pos) > per_node:   # the last ones (nearest the frontier) and a sample of the rest
                pos = np.unique(np.concatenate([pos[-per_node // 2:], rng.choice(pos, per_node // 2)]))
            for i in pos:
                v = value(q, int(i), m)
                later = [value(q, int(i), m2) for m2 in (m + 1, m + 7) if m2 <= n]
                later.append(value(q, int(i), n, full_next))
                if v == U or any(w != v for w in later):
                    bad.append((m, q, int(i), v, later))
                    break
    return bad


CASES = [
    (W.immigration_death, "F[0,10](G[1,2](X>=65))", 1500),
    (W.immigration_death, "G[0,10](X<=60 | F[1,2](X>=70))", 1500),
    (W.isomerization, "X[0,0.1](X[0,0.1](A<=48))", 1500),
    (W.immigration_death, "(F[0,1](X>=5)) U[0,5] (X>=30)", 1500),
    (W.immigration_death, "F[0,3](F[0,2](F[0,1](X>=40)))", 1500),
    (W.isomerization, "G[0,1](F[0,0.5](A>=28)) & G[0,1](F[0,0.5](B>=12)) & G[0,1](F[0,1](A<=45))", 1500),
    (W.immigration_death, "F[5,60](X[0,0.2](X>=115) & G[0,1](X>=105))", 1500),
    (W.immigration_death, "(G[0,2](X<=118)) U[1,50] (F[0,1](X>=116))", 1500),
    (W.immigration_death, "G[10,60](F[1,3](X>=85))", 1500),
    (W.michaelis_menten, "F[0,60]((S<=300) & F[1,5](P>=600))", 3000),
]
PREFIXES = (2, 16, 32, 64, 160, 400, 1000)


def _trace(make, steps, idx):
    net = make()
    states, times, _, absorbed = oracle.path(net, idx, steps, seed=1, model_id=3)
    return net, states, times, absorbed


@pytest.mark.parametrize("make,text,steps", CASES, ids=[c[1] for c in CASES])
def test_final_positions_keep_their_values(make, text, steps):
    rng = np.random.default_rng(3)
    for idx in (0, 7):
        net, states, times, absorbed = _trace(make, steps, idx)
        f = oracle.parse(text, net)
        bad = violations(f, states, times, absorbed, PREFIXES, rng=rng)
        assert not bad, (text, idx, bad[:3])


def test_random_formulas_final_positions():
    """The rule on 40 random nested formulas (each on its own trajectory)."""
    import random
    r = random.Random(12)
    rng = np.random.default_rng(5)
    for q in range(40):
        text = random_formula(r)
        net, states, times, absorbed = _trace(W.immigration_death, 700, q)
        f = oracle.parse(text, net)
        bad = violations(f, states, times, absorbed, (2, 16, 64, 200, 500), per_node=20, rng=rng)
        assert not bad, (text, q, bad[:3])


@pytest.mark.parametrize("mutant,make,text", [
    ("next", W.isomerization, "X[0,0.1](X[0,0.1](A<=48))"),
    ("until-operands", W.immigration_death, "F[0,3](F[0,2](F[0,1](X>=40)))"),
    ("until-window", W.immigration_death, "G[0,10](X<=60 | F[1,2](X>=70))"),
])
def test_planted_rule_mistakes_are_caught(mutant, make, text):
    """Each mistake makes the rule claim a position whose value still changes
    (for the window: times are entered exactly on a grid here, so that a
    position exactly hi after state i occurs)."""
    rng = np.random.default_rng(4)
    found = False
    for idx in range(6):
        net, states, times, absorbed = _trace(make, 1500, idx)
        if mutant == "until-window":
            times = np.round(times * 4.0) / 4.0   # entries on a quarter grid (still non-decreasing)
        f = oracle.parse(text, net)
        if violations(f, states, times, absorbed, PREFIXES, mutant=mutant, rng=rng):
            # on the same trace the rule itself holds
            assert not violations(f, states, times, absorbed, PREFIXES, rng=np.random.default_rng(4))
            found = True
            break
    assert found, mutant
