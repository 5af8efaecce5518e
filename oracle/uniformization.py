"""Exact transient probabilities on small truncated CTMCs (test infrastructure).

TEST INFRASTRUCTURE ONLY.

These are the "exact" numbers the statistical estimates are checked against,
the role PRISM plays in the paper's experiments (Sec. 5).  Two independent
numerical methods are provided:
  - uniformization: pi(T) = sum_k Poisson(k; qT) pi(0) P^k, P = I + Q/q;
  - the matrix exponential pi(T) = pi(0) expm(Q T) (scipy).

For a time-bounded until p1 U^[0,T] p2 with state predicates p1, p2, the
probability is that of the chain in which every p2-state is an absorbing
success and every state with neither p1 nor p2 is an absorbing failure,
being in a success state at time T.  F^[0,T] p = tt U^[0,T] p and
G^[0,T] p = 1 - P(F^[0,T] not p).
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np
import scipy.linalg
import scipy.sparse as sp
from scipy.special import gammaln


def _propensity(net, j, x):
    ra, rb = int(net.reactants[j][0]), int(net.reactants[j][1])
    c = float(net.rate[j])
    if ra < 0 and rb < 0:
        return c
    if ra < 0:
        ra, rb = rb, -1
    if rb < 0:
        return c * x[ra]
    if ra == rb:
        return c * x[ra] * (x[ra] - 1) / 2.0
    return c * x[ra] * x[rb]


def enumerate_chain(net, x0, upper, absorbing=lambda x: False):
    """Breadth-first enumeration of states reachable from x0 with every count
    <= upper[s]; transitions leaving the box are dropped (probability mass
    that leaves is lost, so results are lower bounds unless the box is
    closed).  Returns (states list, index dict, sparse generator Q)."""
    x0 = tuple(int(v) for v in x0)
    index = {x0: 0}
    states = [x0]
    rows, cols, vals = [], [], []
    diag = []
    todo = deque([x0])
    while todo:
        x = todo.popleft()
        i = index[x]
        out = 0.0
        if not absorbing(x):
            for j in range(len(net.rate)):
                a = _propensity(net, j, x)
                if a <= 0.0:
                    continue
                y = list(x)
                for q in range(4):
                    s = int(net.chg_idx[j][q])
                    if s >= 0:
                        y[s] += int(net.chg_val[j][q])
                y = tuple(y)
                if any(v < 0 for v in y):
                    continue
                out += a
                if any(y[s] > upper[s] for s in range(len(y))):
                    continue
                if y not in index:
                    index[y] = len(states)
                    states.append(y)
                    todo.append(y)
                rows.append(i)
                cols.append(index[y])
                vals.append(a)
        diag.append((i, -out))
    n = len(states)
    for i, d in diag:
        rows.append(i)
        cols.append(i)
        vals.append(d)
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return states, index, Q


def transient_uniformization(Q, pi0, T, tol=1e-15):
    """pi(T) by uniformization with Poisson weights taken in log space."""
    q = float(np.max(-Q.diagonal())) * 1.02 + 1e-12
    P = sp.identity(Q.shape[0], format="csr") + Q / q
    lam = q * T
    kmax = int(lam + 12.0 * math.sqrt(lam + 1.0) + 50)
    v = np.asarray(pi0, dtype=np.float64).copy()
    acc = np.zeros_like(v)
    PT = P.T.tocsr()
    for k in range(kmax + 1):
        w = math.exp(k * math.log(lam) - lam - gammaln(k + 1)) if lam > 0 else (1.0 if k == 0 else 0.0)
        if w > tol * 1e-3 or k < lam:
            acc += w * v
        v = PT @ v
    return acc


def transient_expm(Q, pi0, T):
    return np.asarray(pi0, dtype=np.float64) @ scipy.linalg.expm(Q.toarray() * T)


def until_probability(net, p1, p2, T, upper, method="uniformization"):
    """P(p1 U^[0,T] p2) from x0 on the box count <= upper (p1, p2: state -> bool)."""
    x0 = tuple(int(v) for v in net.x0)
    if p2(x0):
        return 1.0
    if not p1(x0):
        return 0.0
    absorbing = lambda x: p2(x) or not p1(x)
    states, index, Q = enumerate_chain(net, x0, upper, absorbing)
    pi0 = np.zeros(len(states))
    pi0[0] = 1.0
    if method == "expm":
        pi = transient_expm(Q, pi0, T)
    else:
        pi = transient_uniformization(Q, pi0, T)
    succ = np.array([1.0 if p2(x) else 0.0 for x in states])
    return float(pi @ succ)


def marginal(net, T, upper, method="expm"):
    """Distribution of the state at time T: (states, probabilities)."""
    x0 = tuple(int(v) for v in net.x0)
    states, index, Q = enumerate_chain(net, x0, upper)
    pi0 = np.zeros(len(states))
    pi0[0] = 1.0
    pi = transient_expm(Q, pi0, T) if method == "expm" else transient_uniformization(Q, pi0, T)
    return states, pi
