"""Pins for the Wilson formulas and the iterative sample-size rule (Sec. 3.3).

- Table 3's printed intervals and conservative sample size (golden fixture);
- the "up to 88%" reduction claimed for Fig. 3 (reached at p = 0 and p = 1);
- the closed form of eq. 4 at p = 1: z^2 (1/(2 eps) - 1);
- the algebraic link between eqs. 3 and 4: at n = eq.4(p) the half-width of
  eq. 3 with p_hat = p is exactly eps;
- z against mpmath's inverse error function;
- coverage of the iterative procedure on Bernoulli streams.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import wilson


def _table3(golden_dir):
    with open(os.path.join(golden_dir, "table3_wilson.json")) as fh:
        return json.load(fh)


def test_z_values():
    """Standard normal quantiles z_{1-alpha/2} of the decimal confidences
    (tabulated to 16 digits) and scipy's independent ndtri.  The confidence
    reaches z_value as the nearest double, so the tolerance allows for that
    input rounding (dz/dc times half an ulp of c)."""
    from scipy.special import ndtri
    table = {0.95: 1.9599639845400542, 0.99: 2.5758293035489008, 0.999: 3.2905267314918948,
             0.9999: 3.8905918864130940}
    for c, zt in table.items():
        z = wilson.z_value(c)
        slope = math.sqrt(math.pi / 2) * math.exp(zt * zt / 2)
        tol = slope * math.ulp(c) + 2 * math.ulp(zt)
        assert abs(z - zt) <= tol, (c, z, zt)
        assert abs(z - float(ndtri(0.5 + 0.5 * c))) <= 4 * tol


def test_table3_intervals(golden_dir):
    t3 = _table3(golden_dir)
    z = wilson.z_value(t3["confidence"])
    for row in t3["intervals"]:
        lo, hi = wilson.wilson_interval(row["successes"], row["n"], z)
        # printed values are truncated/rounded at their last printed digit
        dl = 10.0 ** -(len(repr(row["printed_lo"]).split(".")[1]))
        dh = 10.0 ** -(len(repr(row["printed_hi"]).split(".")[1]))
        assert abs(lo - row["printed_lo"]) <= dl, (row, lo)
        assert abs(hi - row["printed_hi"]) <= dh, (row, hi)
        if row["printed_p"] is not None:
            assert abs(row["successes"] / row["n"] - row["printed_p"]) <= 1e-5


def test_conservative_sample_size(golden_dir):
    t3 = _table3(golden_dir)
    z = wilson.z_value(t3["confidence"])
    assert wilson.wilson_sample(0.5, t3["eps"], z) == t3["conservative_n"]["value"]


def test_iterative_reduction_claim(golden_dir):
    t3 = _table3(golden_dir)
    z = wilson.z_value(t3["confidence"])
    eps = t3["eps"]
    cons = wilson.wilson_sample(0.5, eps, z)
    for always in (0, 1):
        res = wilson.iterative_wilson(lambda lo, hi: always * (hi - lo), eps, z)
        n = res[3]
        assert n == 304
        assert math.floor(100 * (1 - n / cons)) == t3["reduction_claim"]["percent"]


def test_first_batch_closed_form():
    for eps, conf in ((0.025, 0.99), (0.01, 0.95), (0.005, 0.9999)):
        z = wilson.z_value(conf)
        closed = z * z * (1.0 / (2.0 * eps) - 1.0)
        assert wilson.wilson_sample_value(1.0, eps, z) == pytest.approx(closed, rel=1e-12)
        assert wilson.wilson_sample_value(0.0, eps, z) == pytest.approx(closed, rel=1e-12)
    z95 = wilson.z_value(0.95)
    assert wilson.wilson_sample(1.0, 0.01, z95) == 189
    assert wilson.wilson_sample(1.0, 0.025, wilson.z_value(0.99)) == 127


def test_all_false_stream_95():
    z = wilson.z_value(0.95)
    p, lo, hi, n, yes, bounds = wilson.iterative_wilson(lambda a, b: 0, 0.01, z)
    assert (p, n, yes, bounds) == (0.0, 454, 0, [189, 454])
    assert lo == 0.0 and hi == pytest.approx(0.0083904, abs=1e-7)
    assert wilson.wilson_sample(0.5, 0.01, z) == 9600


def test_eq3_eq4_identity():
    """Squaring the half-width of eq. 3 and solving for n gives eq. 4."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        p = float(rng.uniform(0, 1))
        eps = float(rng.uniform(0.002, 0.1))
        z = float(rng.uniform(1.0, 4.0))
        n = wilson.wilson_sample_value(p, eps, z)
        if n <= 1:
            continue
        z2 = z * z
        half = z * math.sqrt(p * (1 - p) / n + z2 / (4 * n * n)) / (1 + z2 / n)
        assert half == pytest.approx(eps, rel=1e-9)


def test_sample_size_shape():
    z = wilson.z_value(0.99)
    ps = np.linspace(0, 1, 11)
    ns = [wilson.wilson_sample_value(float(p), 0.025, z) for p in ps]
    for k in range(5):
        assert ns[k] == pytest.approx(ns[10 - k], rel=1e-12)   # symmetric in p <-> 1-p
        assert ns[k] < ns[k + 1]                               # maximal at 0.5


def test_rounding_towards_half():
    assert wilson.rounded_estimate(0.2, 0.01) == pytest.approx(0.21)
    assert wilson.rounded_estimate(0.8, 0.01) == pytest.approx(0.79)
    assert wilson.rounded_estimate(0.495, 0.01) == 0.5
    assert wilson.rounded_estimate(0.505, 0.01) == 0.5
    assert wilson.rounded_estimate(0.495, 0.01, literal=True) == pytest.approx(0.505)
    assert wilson.rounded_estimate(0.502, 0.01, literal=True) == pytest.approx(0.492)


@pytest.mark.parametrize("p", [0.1, 0.3, 0.5])
def test_iterative_coverage(p):
    rng = np.random.default_rng(int(p * 100))
    z = wilson.z_value(0.95)
    cover = 0
    reps = 300
    for _ in range(reps):
        draws = rng.random(20000) < p
        csum = np.concatenate([[0], np.cumsum(draws)])
        ph, lo, hi, n, yes, bounds = wilson.iterative_wilson(lambda a, b: int(csum[b] - csum[a]), 0.05, z)
        cover += lo <= p <= hi
        assert hi - lo <= 2 * 0.05 + 1e-3
    assert cover / reps >= 0.91
