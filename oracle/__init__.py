"""CPU oracle for on-the-fly statistical model checking (test infrastructure).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the GPU library
(paper_0912_2551_amd); the two meet only through the seeded input generators
in paper_0912_2551_amd/workloads.py, which hold none of the method's
arithmetic.

The SSA, the three-valued BLTLc semantics and the on-the-fly stopping rule are
in smc_oracle.c (built to liboracle.so by __graft_entry__.build(), or on first
use here); the Wilson formulas are in wilson.py, the BLTLc parser in bltlc.py,
exact transient probabilities in uniformization.py.

A network is any object with attributes x0 [S], rate [M], reactants [M,2],
chg_idx [M,4], chg_val [M,4] and names [S] (numpy-convertible).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import bltlc, wilson

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

VERDICT_BIT = 1
R_STATE, R_TIME, R_ABSORB, R_CAP, R_TMAX = range(5)


def compile_oracle(force: bool = False) -> str:
    """Compile smc_oracle.c with gcc (-O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    """The compiled oracle.  ORACLE_LIB_OVERRIDE names another build of it to
    load instead: the pin-strength test runs the pins against copies with a
    planted mistake."""
    global _lib
    if _lib is None:
        override = os.environ.get("ORACLE_LIB_OVERRIDE")
        if override:
            _lib = ctypes.CDLL(override)
        else:
            compile_oracle()
            _lib = ctypes.CDLL(_LIB)
        _lib.oracle_log.restype = ctypes.c_double
        _lib.oracle_log.argtypes = [ctypes.c_double]
        _lib.oracle_path.restype = ctypes.c_int64
        _lib.oracle_eval.restype = ctypes.c_int
        _lib.oracle_run.restype = ctypes.c_int
    return _lib


def set_plain_scan(on: bool) -> None:
    """Evaluate until by scanning every position, as its definition reads
    (True), or jump over positions that cannot change the scan (False, the
    default; same values, linear instead of quadratic time for nested
    untils)."""
    lib().oracle_set_plain_scan(ctypes.c_int(1 if on else 0))


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def log(x: float) -> float:
    return lib().oracle_log(float(x))


def uniforms(r):
    rr = np.asarray(r, dtype=np.uint32)
    out = np.zeros(2, dtype=np.float64)
    lib().oracle_uniforms(_p(rr, ctypes.c_uint32), _p(out, ctypes.c_double))
    return float(out[0]), float(out[1])


# ---------------------------------------------------------------------------
# networks and formulas
# ---------------------------------------------------------------------------
class _Net:
    def __init__(self, net):
        self.x0 = _i32(net.x0)
        self.rate = _f64(net.rate)
        self.reactants = _i32(net.reactants).reshape(-1, 2)
        self.chg_idx = _i32(net.chg_idx).reshape(-1, 4)
        self.chg_val = _i32(net.chg_val).reshape(-1, 4)
        self.S = int(self.x0.shape[0])
        self.M = int(self.rate.shape[0])
        self.names = list(getattr(net, "names", [f"X{k}" for k in range(self.S)]))

    def args(self):
        return (ctypes.c_int32(self.S), ctypes.c_int32(self.M), _p(self.x0, ctypes.c_int32),
                _p(self.rate, ctypes.c_double), _p(self.reactants, ctypes.c_int32),
                _p(self.chg_idx, ctypes.c_int32), _p(self.chg_val, ctypes.c_int32))


class _Form:
    def __init__(self, f: bltlc.Formula):
        self.f = f
        self.type = _i32(f.type)
        self.a = _i32(f.a)
        self.b = _i32(f.b)
        self.lo = _f64(f.lo)
        self.hi = _f64(f.hi)
        self.pred = _i32(f.pred)
        n = max(len(f.pred_op), 1)
        self.pred_op = _i32(f.pred_op or [0])
        self.lhs_off = _i32(f.lhs_off or [0])
        self.lhs_len = _i32(f.lhs_len or [0])
        self.rhs_off = _i32(f.rhs_off or [0])
        self.rhs_len = _i32(f.rhs_len or [0])
        self.prog_op = _i32(f.prog_op or [0])
        self.prog_arg = _f64(f.prog_arg or [0.0])
        self.n_preds = len(f.pred_op) if f.pred_op else 0
        del n

    def args(self):
        return (ctypes.c_int32(self.f.n_nodes), ctypes.c_int32(self.f.root),
                _p(self.type, ctypes.c_int32), _p(self.a, ctypes.c_int32), _p(self.b, ctypes.c_int32),
                _p(self.lo, ctypes.c_double), _p(self.hi, ctypes.c_double),
                _p(self.pred, ctypes.c_int32), ctypes.c_int32(self.n_preds),
                _p(self.pred_op, ctypes.c_int32), _p(self.lhs_off, ctypes.c_int32),
                _p(self.lhs_len, ctypes.c_int32), _p(self.rhs_off, ctypes.c_int32),
                _p(self.rhs_len, ctypes.c_int32), _p(self.prog_op, ctypes.c_int32),
                _p(self.prog_arg, ctypes.c_double))


def parse(text: str, net) -> bltlc.Formula:
    return bltlc.parse(text, _Net(net).names)


def default_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def horizon(f: bltlc.Formula, node: int | None = None) -> float:
    """Time span of the path that can influence the formula: a predicate
    looks at one state; X^I and U^I reach sup I beyond their operands."""
    k = f.root if node is None else node
    t = f.type[k]
    if t in (bltlc.N_TRUE, bltlc.N_FALSE, bltlc.N_PRED):
        return 0.0
    if t == bltlc.N_NOT:
        return horizon(f, f.a[k])
    if t in (bltlc.N_AND, bltlc.N_OR):
        return max(horizon(f, f.a[k]), horizon(f, f.b[k]))
    if t == bltlc.N_NEXT:
        return f.hi[k] + horizon(f, f.a[k])
    return f.hi[k] + max(horizon(f, f.a[k]), horizon(f, f.b[k]))


def trajectories(net, formula, first: int, count: int, seed: int = 1, model_id: int = 0,
                 max_events: int = 0, t_max: float = math.inf, threads: int | None = None):
    """Per-trajectory (events, verdict, reason) for indices [first, first+count)."""
    n = _Net(net)
    f = _Form(formula if isinstance(formula, bltlc.Formula) else bltlc.parse(formula, n.names))
    if math.isinf(horizon(f.f)) and math.isinf(t_max) and not max_events:
        raise ValueError("an unbounded formula needs t_max or max_events")
    ev = np.zeros(count, dtype=np.uint32)
    vd = np.zeros(count, dtype=np.uint8)
    rs = np.zeros(count, dtype=np.uint8)
    if count == 0:
        return ev, vd, rs
    rc = lib().oracle_run(*n.args(), *f.args(), ctypes.c_uint64(seed), ctypes.c_uint32(model_id),
                          ctypes.c_uint32(max_events), ctypes.c_double(t_max),
                          ctypes.c_uint64(first), ctypes.c_uint64(count),
                          ctypes.c_int32(threads or default_threads()),
                          _p(ev, ctypes.c_uint32), _p(vd, ctypes.c_uint8), _p(rs, ctypes.c_uint8))
    if rc != 0:
        raise RuntimeError("oracle trajectory failed")
    return ev, vd, rs


def path(net, idx: int, n_steps: int, seed: int = 1, model_id: int = 0):
    """Raw SSA path of trajectory idx for up to n_steps steps.

    Returns (states [n, S], times [n], a0 [n-1 or n], absorbed): states and
    their entry times; a0[q] is the total propensity in state q; when the
    path reached an absorbing state early, absorbed is True and a0[-1] == 0."""
    n = _Net(net)
    states = np.zeros((n_steps + 1, n.S), dtype=np.int32)
    times = np.zeros(n_steps + 2, dtype=np.float64)
    a0 = np.zeros(n_steps + 1, dtype=np.float64)
    got = lib().oracle_path(*n.args(), ctypes.c_uint64(seed), ctypes.c_uint32(model_id),
                            ctypes.c_uint64(idx), ctypes.c_int64(n_steps),
                            _p(states, ctypes.c_int32), _p(times, ctypes.c_double),
                            _p(a0, ctypes.c_double))
    absorbed = got <= n_steps
    return states[:got], times[:got], (a0[:got] if absorbed else a0[:n_steps]), absorbed


def sample_state(net, T: float, first: int, count: int, seed: int = 1, model_id: int = 0):
    """sigma @ T for trajectories [first, first+count): array [count, S]."""
    n = _Net(net)
    out = np.zeros((count, n.S), dtype=np.int32)
    lib().oracle_sample_state(*n.args(), ctypes.c_uint64(seed), ctypes.c_uint32(model_id),
                              ctypes.c_double(T), ctypes.c_uint64(first), ctypes.c_uint64(count),
                              _p(out, ctypes.c_int32))
    return out


def eval_prefix(formula: bltlc.Formula, states, times, next_time=None) -> int:
    """Three-valued value (0 F, 1 T, 2 unknown) of the formula at position 0
    of the prefix states[0..n-1] with entry times times[0..n-1]; next_time is
    the time the last state is left (math.inf: absorbing; None: unknown)."""
    st = _i32(states)
    if st.ndim == 1:
        st = st.reshape(-1, 1)
    n = st.shape[0]
    t = np.zeros(n + 1, dtype=np.float64)
    t[:n] = np.asarray(times, dtype=np.float64)[:n]
    known = next_time is not None
    if known:
        t[n] = next_time
    f = _Form(formula)
    return lib().oracle_eval(ctypes.c_int32(st.shape[1]), *f.args(), ctypes.c_int64(n),
                             ctypes.c_int32(1 if known else 0), _p(st, ctypes.c_int32),
                             _p(t, ctypes.c_double))


def estimate(net, formula, confidence: float = 0.95, eps: float = 0.01, fixed_n: int = 0,
             seed: int = 1, model_id: int = 0, max_events: int = 0, t_max: float = math.inf,
             conservative: bool = False, literal: bool = False, z: float | None = None,
             threads: int | None = None):
    """Full estimate: fixed N, or the iterative Wilson rule of Fig. 2.

    Returns a dict with p_hat, lo, hi, n, successes, events, truncated, bounds."""
    n = _Net(net)
    f = formula if isinstance(formula, bltlc.Formula) else bltlc.parse(formula, n.names)
    zz = wilson.z_value(confidence) if z is None else float(z)
    stats = {"events": 0, "truncated": 0}

    def count_yes(lo, hi):
        ev, vd, rs = trajectories(net, f, lo, hi - lo, seed, model_id, max_events, t_max, threads)
        stats["events"] += int(ev.sum(dtype=np.uint64))
        stats["truncated"] += int((rs == R_CAP).sum())
        return int(vd.sum())

    if fixed_n:
        yes = count_yes(0, fixed_n)
        lo, hi = wilson.wilson_interval(yes, fixed_n, zz)
        return dict(p_hat=yes / fixed_n, lo=lo, hi=hi, n=fixed_n, successes=yes,
                    bounds=[fixed_n], **stats)
    p_hat, lo, hi, ntot, yes, bounds = wilson.iterative_wilson(count_yes, eps, zz, conservative,
                                                               literal)
    return dict(p_hat=p_hat, lo=lo, hi=hi, n=ntot, successes=yes, bounds=bounds, **stats)
