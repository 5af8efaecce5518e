"""Pins for the oracle's formula probabilities against exact values.

The exact values come from the transient solution of the truncated CTMC
(uniformization and the matrix exponential, which must agree with each other),
playing the role PRISM plays in the paper's accuracy experiment (Sec. 5,
Fig. 6 and Table 3): the oracle's estimate must contain the exact value in
its 99.9% Wilson interval (eq. 3).  The Next operator is checked against the
closed form that follows from eqs. 2a/2b.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.uniformization as U
from oracle import wilson
from paper_0912_2551_amd import workloads as W

Z999 = wilson.z_value(0.999)


def estimate_contains(net, text, exact, n, seed=1):
    f = oracle.parse(text, net)
    ev, vd, rs = oracle.trajectories(net, f, 0, n, seed=seed)
    lo, hi = wilson.wilson_interval(int(vd.sum()), n, Z999)
    assert lo <= exact <= hi, (text, vd.mean(), exact, lo, hi)
    return vd.mean(), ev


def test_c1_against_uniformization():
    net = W.immigration_death()
    exact = U.until_probability(net, lambda x: True, lambda x: x[0] >= 120, 100.0, [400])
    exact2 = U.until_probability(net, lambda x: True, lambda x: x[0] >= 120, 100.0, [400], "expm")
    assert abs(exact - exact2) < 1e-10
    assert abs(exact - 0.507334) < 5e-6
    p, ev = estimate_contains(net, W.C1_FORMULA, exact, 20000)
    assert 1300 < ev.mean() < 1700


@pytest.mark.parametrize("T", [25.0, 50.0])
def test_c1_time_sweep(T):
    net = W.immigration_death()
    exact = U.until_probability(net, lambda x: True, lambda x: x[0] >= 120, T, [400])
    estimate_contains(net, f"F[0,{T:g}](X>=120)", exact, 20000, seed=2)


def test_until_isomerization():
    net = W.isomerization(1.0, 0.5, 50)
    exact = U.until_probability(net, lambda x: x[1] <= 30, lambda x: x[0] <= 20, 1.5, [50, 50])
    exact2 = U.until_probability(net, lambda x: x[1] <= 30, lambda x: x[0] <= 20, 1.5, [50, 50], "expm")
    assert abs(exact - exact2) < 1e-10
    assert 0.05 < exact < 0.95
    estimate_contains(net, "(B<=30) U[0,1.5] (A<=20)", exact, 20000)


def test_until_two_independent_species():
    """The left operand can fail before the right one holds (Y and X evolve
    independently), so the until's 'p1 at every earlier state' matters here:
    without it the probability would be that of F, 0.63 instead of 0.43."""
    net = W.from_reactions(["X", "Y"], [0, 0], [([], ["X"], 1.0), (["X"], [], 0.1),
                                                  ([], ["Y"], 1.0), (["Y"], [], 0.1)], "two immigration-death")
    exact = U.until_probability(net, lambda x: x[1] <= 3, lambda x: x[0] >= 4, 5.0, [40, 40])
    exact2 = U.until_probability(net, lambda x: x[1] <= 3, lambda x: x[0] >= 4, 5.0, [40, 40], "expm")
    fin = U.until_probability(net, lambda x: True, lambda x: x[0] >= 4, 5.0, [40, 40])
    assert abs(exact - exact2) < 1e-10
    assert 0.05 < exact < 0.95 and fin - exact > 0.1
    estimate_contains(net, "(Y<=3) U[0,5] (X>=4)", exact, 20000)


def test_globally_isomerization():
    net = W.isomerization(1.0, 0.5, 50)
    fin = U.until_probability(net, lambda x: True, lambda x: x[0] < 22, 1.0, [50, 50])
    exact = 1.0 - fin
    assert 0.05 < exact < 0.95
    estimate_contains(net, "G[0,1](A>=22)", exact, 20000, seed=3)


@pytest.mark.parametrize("lo,hi", [(0.0, 0.002), (0.001, 0.002)])
def test_next_closed_form(lo, hi):
    net = W.michaelis_menten()
    net.x0[:] = [90, 990, 10, 0]
    a = np.array([0.01 * 90 * 990, 0.1 * 10, 0.1 * 10])
    a0 = a.sum()
    exact = a[0] / a0 * (math.exp(-a0 * lo) - math.exp(-a0 * hi))
    estimate_contains(net, f"X[{lo:g},{hi:g}](ES>=11)", exact, 20000, seed=4)


def test_c2_is_identically_false():
    """E + ES = 100 and S + ES + P = 1000: S <= 200 needs P >= 700, so an
    earlier state has P = 500 with S = 500 - ES >= 400 > 200, where P < 500
    fails.  The until conjunct is therefore false on every path."""
    net = W.michaelis_menten()
    ev, vd, rs = oracle.trajectories(net, oracle.parse(W.C2_FORMULA, net), 0, 20000)
    assert vd.sum() == 0
    assert (rs == oracle.R_STATE).all()
    assert 80 < ev.mean() < 120
