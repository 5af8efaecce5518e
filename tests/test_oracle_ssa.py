"""Pins for the oracle's direct-method SSA (Sec. 2.2, eqs. 1, 2a, 2b).

Distributional checks against closed forms and an independent numerical
solution of the master equation:
- immigration-death 0 -> X (k), X -> 0 (mu X) from 0: X(T) ~ Poisson((k/mu)(1 - e^{-mu T}));
- isomerization A <-> B from N0 in A: A(T) ~ Binomial(N0, q), q = c2/(c1+c2) + c1/(c1+c2) e^{-(c1+c2) T};
- homodimerization A + A -> B and A + B -> C against the matrix exponential of the
  generator (checks the x(x-1)/2 and x_a x_b combinatorial factors);
- first step from a fixed state: reaction j with probability a_j/a0 and sojourn
  time Exp(a0), the factorisation of eq. 1 into eqs. 2a and 2b.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import oracle.uniformization as U
from paper_0912_2551_amd import workloads as W


def chi2_pvalue(samples, support, pmf):
    """Pearson chi-square over bins merged until every expected count >= 5."""
    n = len(samples)
    counts = {v: 0 for v in support}
    other = 0
    for v in samples:
        if v in counts:
            counts[v] += 1
        else:
            other += 1
    obs, exp = [], []
    acc_o, acc_e = 0, 0.0
    for v, p in zip(support, pmf):
        acc_o += counts[v]
        acc_e += n * p
        if acc_e >= 5:
            obs.append(acc_o)
            exp.append(acc_e)
            acc_o, acc_e = 0, 0.0
    rest = n - sum(exp)
    obs.append(acc_o + other)
    exp.append(acc_e + max(rest - acc_e, 0.0))
    if exp[-1] < 5 and len(exp) > 1:
        obs[-2] += obs[-1]
        exp[-2] += exp[-1]
        obs, exp = obs[:-1], exp[:-1]
    exp = np.asarray(exp) * (n / np.sum(exp))
    return stats.chisquare(obs, exp).pvalue


@pytest.mark.parametrize("T", [5.0, 40.0])
def test_immigration_death_poisson(T):
    net = W.immigration_death(10.0, 0.1, 0)
    xs = oracle.sample_state(net, T, 0, 20000, seed=12)[:, 0]
    lam = (10.0 / 0.1) * (1.0 - math.exp(-0.1 * T))
    support = list(range(0, int(lam + 12 * math.sqrt(lam) + 20)))
    assert chi2_pvalue(list(xs), support, stats.poisson.pmf(support, lam)) > 1e-4
    assert abs(xs.mean() - lam) < 5 * math.sqrt(lam / len(xs))


@pytest.mark.parametrize("T", [0.3, 2.0])
def test_isomerization_binomial(T):
    c1, c2, n0 = 1.0, 0.5, 50
    net = W.isomerization(c1, c2, n0)
    xs = oracle.sample_state(net, T, 0, 20000, seed=13)
    assert (xs.sum(axis=1) == n0).all()
    q = c2 / (c1 + c2) + c1 / (c1 + c2) * math.exp(-(c1 + c2) * T)
    support = list(range(n0 + 1))
    assert chi2_pvalue(list(xs[:, 0]), support, stats.binom.pmf(support, n0, q)) > 1e-4


@pytest.mark.parametrize("which", ["homodimer", "heterodimer"])
def test_bimolecular_against_master_equation(which):
    if which == "homodimer":
        net = W.dimerization(0.02, 40)
        T = 2.0
    else:
        net = W.from_reactions(["A", "B", "C"], [30, 20, 0], [(["A", "B"], ["C"], 0.01)], "AB")
        T = 3.0
    states, pi = U.marginal(net, T, [100] * net.S)
    xs = oracle.sample_state(net, T, 0, 20000, seed=14)
    key = {tuple(s): k for k, s in enumerate(states)}
    samples = [key[tuple(int(v) for v in row)] for row in xs]
    assert chi2_pvalue(samples, list(range(len(states))), pi) > 1e-4
    # A wrong combinatorial factor would shift the mean far outside this band.
    mean_exact = float(sum(p * s[0] for s, p in zip(states, pi)))
    assert abs(xs[:, 0].mean() - mean_exact) < 0.05 * max(mean_exact, 1.0)


def test_first_step_factorisation():
    net = W.michaelis_menten()
    net.x0[:] = [90, 990, 10, 0]
    a = np.array([0.01 * 90 * 990, 0.1 * 10, 0.1 * 10])
    a0 = a.sum()
    n = 30000
    picks = np.zeros(3, dtype=np.int64)
    taus = np.zeros(n)
    for i in range(n):
        st, tm, a0s, _ = oracle.path(net, i, 1, seed=21)
        d = st[1] - st[0]
        if d[2] == 1:
            picks[0] += 1
        elif d[1] == 1:
            picks[1] += 1
        else:
            picks[2] += 1
        taus[i] = tm[1]
        assert a0s[0] == pytest.approx(a0, rel=1e-15)
    assert stats.chisquare(picks, n * a / a0).pvalue > 1e-4
    assert stats.kstest(taus, "expon", args=(0, 1.0 / a0)).pvalue > 1e-4


def test_conservation_laws_michaelis_menten():
    net = W.michaelis_menten()
    st, tm, _, _ = oracle.path(net, 3, 5000)
    assert (st[:, 0] + st[:, 2] == 100).all()
    assert (st[:, 1] + st[:, 2] + st[:, 3] == 1000).all()
    assert (st >= 0).all()
    assert (np.diff(tm) >= 0).all()
