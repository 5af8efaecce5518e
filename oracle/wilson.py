"""Wilson score interval and the iterative sample-size rule (oracle side).

TEST INFRASTRUCTURE ONLY.

Sec. 3.3 of the paper:
  eq. 3  Wilson_interval(p, n, alpha) = [L, U]
         = (p + z^2/(2n) -/+ z sqrt(p(1-p)/n + z^2/(4n^2))) / (1 + z^2/n)
  eq. 4  Wilson_sample(p, eps, alpha) = N
         N >= z^2 (p(1-p) - 2 eps^2 + sqrt(p^2(1-p)^2 + 4 eps^2 (p - 0.5)^2)) / (2 eps^2)
  Fig. 2 the iterative procedure: start from N = Wilson_sample(1), estimate
         p from all runs so far, move it by eps towards 0.5, recompute the
         sample size and run the difference, until no more runs are needed.
z is the (1 - alpha/2) quantile of the standard normal distribution.

Python floats are IEEE doubles and Python never contracts a*b+c, so the
operation order written here is the order that is executed.
"""
from __future__ import annotations

import math

import mpmath


def z_value(confidence: float) -> float:
    """z_{1-alpha/2} for confidence 1-alpha: the standard normal quantile,
    sqrt(2) erfinv(1 - alpha), evaluated at 40 digits and rounded once."""
    if not (0.0 < confidence < 1.0):
        raise ValueError("confidence must lie in (0, 1)")
    with mpmath.workdps(40):
        return float(mpmath.sqrt(2) * mpmath.erfinv(mpmath.mpf(confidence)))


def wilson_sample_value(p: float, eps: float, z: float) -> float:
    """Right-hand side of eq. 4 before rounding up."""
    pq = p * (1.0 - p)
    e2 = eps * eps
    d = p - 0.5
    rad = pq * pq + (4.0 * e2) * (d * d)
    num = (pq - 2.0 * e2) + math.sqrt(rad)
    return (z * z) * num / (2.0 * e2)


def wilson_sample(p: float, eps: float, z: float) -> int:
    """Smallest integer N satisfying eq. 4."""
    return int(math.ceil(wilson_sample_value(p, eps, z)))


def wilson_interval(successes: int, n: int, z: float):
    """Eq. 3 with p = successes / n, clipped to [0, 1]."""
    if n <= 0:
        return 0.0, 1.0
    nd = float(n)
    p = successes / nd
    z2 = z * z
    center = p + z2 / (2.0 * nd)
    half = z * math.sqrt(p * (1.0 - p) / nd + z2 / ((4.0 * nd) * nd))
    den = 1.0 + z2 / nd
    lo = (center - half) / den
    hi = (center + half) / den
    return max(lo, 0.0), min(hi, 1.0)


def rounded_estimate(p: float, eps: float, literal: bool = False) -> float:
    """Fig. 2: move the estimate by eps towards 0.5.

    The paper adds eps when p <= 0.5 and subtracts it otherwise.  Taken
    literally this can step across 0.5 (p = 0.495 -> 0.505), which gives a
    slightly smaller sample than p' = 0.5 would; by default the step stops at
    0.5, which keeps the stated purpose of the rounding (never an undersized
    sample).  literal=True applies the step exactly as printed.
    """
    if p <= 0.5:
        q = p + eps
        return q if literal else min(q, 0.5)
    q = p - eps
    return q if literal else max(q, 0.5)


def iterative_wilson(count_yes, eps: float, z: float, conservative: bool = False,
                     literal: bool = False, max_batches: int = 1000):
    """Fig. 2.  count_yes(lo, hi) returns the number of TRUE verdicts among
    trajectory indices [lo, hi).  Returns (p_hat, lo, hi, n, successes, bounds)
    where bounds lists the cumulative sample size after every batch."""
    n_tot = 0
    yes = 0
    bounds = []
    n_run = wilson_sample(0.5 if conservative else 1.0, eps, z)
    for _ in range(max_batches):
        yes += count_yes(n_tot, n_tot + n_run)
        n_tot += n_run
        bounds.append(n_tot)
        p_hat = yes / n_tot
        n_prime = wilson_sample(rounded_estimate(p_hat, eps, literal), eps, z)
        n_new = n_prime - n_tot
        if n_new > 0:
            n_run = n_new
            continue
        lo, hi = wilson_interval(yes, n_tot, z)
        return p_hat, lo, hi, n_tot, yes, bounds
    raise RuntimeError("iterative Wilson did not stop")
