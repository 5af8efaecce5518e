"""Pins for the oracle's random-number and logarithm primitives.

- Philox4x32-10 against rocRAND's independent host-callable engine (compiled
  from its header at test time);
- the IEEE-only logarithm against mpmath at 50 digits (<= 1 ulp);
- the 53-bit uniform conversions: exact, in (0,1] and [0,1) respectively.
"""
import math
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("prr") / "prr")
    subprocess.check_call([hipcc, "-O1", os.path.join(HERE, "golden", "rocrand_philox_ref.cpp"),
                           "-o", exe], cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(2024)
    rows = [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF),
            (123, 0, 1, 0, 7, 0), (5, 0, 0xDEADBEEF, 0x01234567, 999999, 3)]
    for _ in range(400):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (1 << 30)
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        rows.append(tuple(int(v) for v in (*c, *k)))
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(rows)
    for r, e in zip(rows, ref):
        got = tuple(int(v) for v in oracle.philox(r[:4], r[4:]))
        assert got == e, (r, got, e)


def test_first_event_follows_the_stream_contract(rocrand_ref):
    """The stream map, end to end: the first event of trajectory idx of a job
    (seed, model) uses the Philox block at counter (0, idx, model, 0) and key
    (seed_lo, seed_hi), u1 from words 0-1 for the holding time and u2 from
    words 2-3 for the channel.  The block comes from rocRAND, ln from mpmath."""
    from paper_0912_2551_amd import workloads as W
    net = W.from_reactions(["X", "Y"], [5, 7], [(["X"], ["Y"], 1.0), (["Y"], ["X"], 0.75), ([], ["X"], 2.0)],
                           "three channels")
    a = [5.0, 5.25, 2.0]                      # propensities at (5, 7); their sums are exact
    S = [5.0, 10.25, 12.25]
    a0 = S[-1]
    jobs = [(1, 0), (0x0000000500000003, 7), (0xFFFFFFFF00000001, 0x0BADCAFE)]
    idxs = list(range(48)) + [1000, 123456, (1 << 30) - 1]
    rows = [(0, i, m, 0, seed & 0xFFFFFFFF, seed >> 32) for seed, m in jobs for i in idxs]
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    words = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(words) == len(rows)
    mpmath.mp.dps = 40
    for r, w in zip(rows, words):
        seed, m, i = r[4] | (r[5] << 32), r[2], r[1]
        u1 = ((w[0] << 21 | w[1] >> 11) + 1) * 2.0**-53
        u2 = (w[2] << 21 | w[3] >> 11) * 2.0**-53
        tau = float(-mpmath.log(mpmath.mpf(u1)) / a0)
        target = u2 * a0
        j = next(k for k in range(3) if S[k] > target)
        states, times, a0s, _ = oracle.path(net, i, 1, seed=seed, model_id=m)
        assert a0s[0] == a0
        assert abs(times[1] - tau) <= 2 * math.ulp(tau), (r, times[1], tau)
        d = tuple(int(v) for v in states[1] - states[0])
        assert d == [(-1, 1), (1, -1), (1, 0)][j], (r, d, j)
    assert a[0] + a[1] + a[2] == a0


def _ulp_error(x):
    mpmath.mp.dps = 50
    exact = mpmath.log(mpmath.mpf(x))
    got = oracle.log(x)
    if exact == 0:
        return 0.0 if got == 0.0 else float("inf")
    ulp = math.ulp(float(exact))
    return float(abs(mpmath.mpf(got) - exact) / ulp)


def test_log_within_one_ulp():
    rng = np.random.default_rng(5)
    xs = [2.0**-53, 1.0 - 2.0**-53, 1.0, 0.5, 0.25, 0.75, math.sqrt(0.5), 1 / math.sqrt(2),
          np.nextafter(math.sqrt(0.5), 0), np.nextafter(math.sqrt(0.5), 1), 0.999, 1e-10, 3.0, 1e300]
    xs += list(rng.integers(1, 2**53, size=3000) * 2.0**-53)
    xs += list(np.exp(rng.uniform(-36, 0, size=1000)))
    worst = 0.0
    for x in xs:
        e = _ulp_error(float(x))
        worst = max(worst, e)
    assert worst <= 1.0, worst
    assert oracle.log(1.0) == 0.0


def test_uniform_conversions_exact():
    u1, u2 = oracle.uniforms([0, 0, 0, 0])
    assert u1 == 2.0**-53 and u2 == 0.0
    u1, u2 = oracle.uniforms([0xFFFFFFFF] * 4)
    assert u1 == 1.0 and u2 == 1.0 - 2.0**-53
    rng = np.random.default_rng(1)
    for _ in range(1000):
        r = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        u1, u2 = oracle.uniforms(r)
        a = (r[0] << 21) | (r[1] >> 11)
        b = (r[2] << 21) | (r[3] >> 11)
        assert u1 == (a + 1) / 2.0**53 and 0.0 < u1 <= 1.0
        assert u2 == b / 2.0**53 and 0.0 <= u2 < 1.0
