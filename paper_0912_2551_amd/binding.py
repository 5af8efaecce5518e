"""Python binding of libsmc (include/smc.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts numpy
arrays and Python values into the C structures and back.  If the library is
not built, or cannot be loaded, calls fail with LibraryMissing: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SMC_LIBRARY may name another build of the same library (tuning experiments).
LIB_PATH = os.environ.get("SMC_LIBRARY") or os.path.join(_HERE, "libsmc.so")

SMC_OK = 0
SMC_E_INVALID = -1
SMC_E_PARSE = -2
SMC_E_UNSUPPORTED = -3
SMC_E_HIP = -4
SMC_E_NOMEM = -5
SMC_E_CANCELLED = -6
SMC_E_TIMEOUT = -7
SMC_CONSERVATIVE_START = 1
SMC_PAPER_ROUNDING = 2
SMC_NO_SPECULATION = 4
SMC_DEVICE_PTRS = 8
SMC_TREE_SUMS = 16
NOALLOC_MAX_JOBS = 64
REASON_STATE, REASON_TIME, REASON_ABSORB, REASON_CAP, REASON_TMAX = range(5)

SPECIALIZE_AUTO, SPECIALIZE_OFF, SPECIALIZE_REQUIRED = 0, 1, 2
KERNEL_GENERIC_SMALL, KERNEL_GENERIC, KERNEL_SPECIALIZED, KERNEL_GENERIC_GROUPED = 0, 1, 2, 3
KERNEL_GENERIC_TREE = 4
KERNEL_GENERIC_TRACE = 5

EXPORTS = [
    "smc_ctx_create", "smc_ctx_destroy", "smc_last_error", "smc_set_watchdog",
    "smc_set_waves_per_cu", "smc_set_specialization", "smc_last_kernel",
    "smc_set_kernel_occupancy", "smc_set_lanes_per_trajectory", "smc_autotune", "smc_autotune_batch",
    "smc_cancel", "smc_device_cus", "smc_net_create",
    "smc_net_set_rates", "smc_net_destroy", "smc_formula_compile", "smc_formula_horizon", "smc_formula_check",
    "smc_formula_destroy", "smc_estimate", "smc_estimate_batch", "smc_estimate_batch_noalloc",
    "smc_trajectories",
    "smc_sample_state", "smc_z_value", "smc_wilson_sample_value", "smc_wilson_sample",
    "smc_wilson_interval", "smc_wilson_next_device", "smc_surrogate_create",
    "smc_surrogate_param_count", "smc_surrogate_set_params", "smc_surrogate_get_params",
    "smc_surrogate_gradients", "smc_surrogate_train", "smc_surrogate_query", "smc_surrogate_calibrate",
    "smc_surrogate_neighbourhood", "smc_surrogate_confirm",
    "smc_surrogate_hull",
    "smc_surrogate_destroy", "smc_convex_hull",
]


class TuneResult(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("specialization", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("events_per_s", ctypes.c_double), ("default_events_per_s", ctypes.c_double)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("seconds", ctypes.c_double), ("default_seconds", ctypes.c_double)]


class LibraryMissing(RuntimeError):
    pass


class SmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsmc error {code}: {msg}")
        self.code = code


class NetDesc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("x0", ctypes.POINTER(ctypes.c_int32)), ("rate", ctypes.POINTER(ctypes.c_double)),
                ("reactants", ctypes.POINTER(ctypes.c_int32)),
                ("change_idx", ctypes.POINTER(ctypes.c_int32)),
                ("change_val", ctypes.POINTER(ctypes.c_int32)),
                ("names", ctypes.POINTER(ctypes.c_char_p))]


class Params(ctypes.Structure):
    _fields_ = [("confidence", ctypes.c_double), ("half_width", ctypes.c_double),
                ("z", ctypes.c_double), ("fixed_n", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("model_id", ctypes.c_uint32), ("max_events", ctypes.c_uint32),
                ("t_max", ctypes.c_double), ("flags", ctypes.c_uint32), ("lanes", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("p_hat", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("n", ctypes.c_uint64), ("successes", ctypes.c_uint64), ("events", ctypes.c_uint64),
                ("truncated", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("wasted", ctypes.c_uint64),
                ("z", ctypes.c_double),
                ("device_seconds", ctypes.c_double), ("status", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float)]


class JobDesc(ctypes.Structure):
    _fields_ = [("net", ctypes.c_void_p), ("formula", ctypes.c_void_p), ("params", Params)]


_lib = None


def lib():
    """Load libsmc.so (built by __graft_entry__.build() or build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        try:
            L = ctypes.CDLL(LIB_PATH)
        except OSError as e:
            raise LibraryMissing(f"cannot load {LIB_PATH}: {e}") from e
        vp, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        sig = {
            "smc_ctx_create": (i32, [i32, vp, ctypes.POINTER(vp)]),
            "smc_ctx_destroy": (None, [vp]),
            "smc_last_error": (ctypes.c_char_p, [vp]),
            "smc_set_watchdog": (i32, [vp, dbl]),
            "smc_set_waves_per_cu": (i32, [vp, i32]),
            "smc_set_specialization": (i32, [vp, i32]),
            "smc_last_kernel": (i32, [vp]),
            "smc_set_kernel_occupancy": (i32, [vp, i32]),
            "smc_set_lanes_per_trajectory": (i32, [vp, i32]),
            "smc_autotune": (i32, [vp, vp, vp, ctypes.POINTER(Params), ctypes.c_uint64, ctypes.POINTER(TuneResult)]),
            "smc_cancel": (None, [vp]),
            "smc_device_cus": (i32, [vp]),
            "smc_net_create": (i32, [vp, ctypes.POINTER(NetDesc), ctypes.POINTER(vp)]),
            "smc_net_set_rates": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
            "smc_net_destroy": (None, [vp]),
            "smc_formula_compile": (i32, [vp, vp, ctypes.c_char_p, ctypes.POINTER(vp)]),
            "smc_formula_horizon": (dbl, [vp]),
            "smc_formula_check": (i32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p), i32,
                                        ctypes.POINTER(dbl), ctypes.c_char_p, ctypes.c_size_t]),
            "smc_formula_destroy": (None, [vp]),
            "smc_estimate": (i32, [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Result)]),
            "smc_estimate_batch": (i32, [vp, ctypes.POINTER(JobDesc), ctypes.c_size_t, ctypes.POINTER(Result)]),
            "smc_autotune_batch": (i32, [vp, ctypes.POINTER(JobDesc), ctypes.c_size_t, ctypes.c_double,
                                         ctypes.POINTER(BatchTuneResult)]),
            "smc_estimate_batch_noalloc": (i32, [vp, ctypes.POINTER(JobDesc), ctypes.c_size_t,
                                                 ctypes.POINTER(Result)]),
            "smc_trajectories": (i32, [vp, vp, vp, ctypes.POINTER(Params), u64, u64, vp, vp]),
            "smc_sample_state": (i32, [vp, vp, ctypes.POINTER(Params), dbl, u64, u64, vp]),
            "smc_z_value": (dbl, [dbl]),
            "smc_wilson_sample_value": (dbl, [dbl, dbl, dbl]),
            "smc_wilson_sample": (u64, [dbl, dbl, dbl]),
            "smc_wilson_interval": (None, [u64, u64, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
            "smc_wilson_next_device": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.c_size_t, dbl, dbl, ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_uint64)]),
            "smc_surrogate_create": (i32, [vp, u64, ctypes.POINTER(vp)]),
            "smc_surrogate_param_count": (ctypes.c_size_t, []),
            "smc_surrogate_set_params": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
            "smc_surrogate_get_params": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
            "smc_surrogate_gradients": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_float), ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
            "smc_surrogate_train": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float), ctypes.c_size_t,
                                          ctypes.POINTER(TrainOpts), ctypes.POINTER(ctypes.c_float)]),
            "smc_surrogate_query": (i32, [vp, vp, ctypes.c_size_t, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_uint32, vp, vp]),
            "smc_surrogate_calibrate": (i32, [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_float)]),
            "smc_surrogate_neighbourhood": (ctypes.c_float, [vp]),
            "smc_surrogate_confirm": (i32, [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_float, ctypes.c_uint32, vp]),
            "smc_surrogate_hull": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
            "smc_surrogate_destroy": (None, [vp]),
            "smc_convex_hull": (i32, [ctypes.POINTER(ctypes.c_float), ctypes.c_size_t,
                                      ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _dptr(t):
    """Device address of an array object (anything with data_ptr(), such as a
    torch tensor), or None."""
    return None if t is None else ctypes.c_void_p(int(t.data_ptr()))


def params(confidence=0.95, half_width=0.01, z=0.0, fixed_n=0, seed=1, model_id=0, max_events=0,
           t_max=math.inf, conservative=False, paper_rounding=False, speculate=True, lanes=0,
           tree_sums=False) -> Params:
    flags = ((SMC_CONSERVATIVE_START if conservative else 0) | (SMC_PAPER_ROUNDING if paper_rounding else 0)
             | (0 if speculate else SMC_NO_SPECULATION) | (SMC_TREE_SUMS if tree_sums else 0))
    return Params(confidence, half_width, z, fixed_n, seed, model_id, max_events, t_max, flags, lanes)


def _torch_runtime_first():
    """torch ships a HIP runtime of its own beside the one this library links.
    Both can serve one process (device pointers pass between them), but only
    if torch's starts first: started after the library's, it finds no
    devices.  So start it, where torch is installed, before the library's
    first HIP call."""
    try:
        import torch
    except ImportError:
        return
    try:
        torch.cuda.init()
    except (RuntimeError, AssertionError):
        pass


class Context:
    """A libsmc context on one HIP device; `stream` may be a torch.cuda.Stream
    (or its integer handle) so that work is ordered with torch's."""

    def __init__(self, device: int = 0, stream=None):
        _torch_runtime_first()
        L = lib()
        handle = None
        if stream is not None:
            handle = ctypes.c_void_p(getattr(stream, "cuda_stream", stream))
        out = ctypes.c_void_p()
        rc = L.smc_ctx_create(device, handle, ctypes.byref(out))
        if rc != SMC_OK:
            raise SmcError(rc, L.smc_last_error(None).decode())
        self.h = out
        self._keep = []

    def _check(self, rc):
        if rc != SMC_OK:
            raise SmcError(rc, lib().smc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().smc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_watchdog(self, seconds: float):
        self._check(lib().smc_set_watchdog(self.h, float(seconds)))

    def set_waves_per_cu(self, w: int):
        self._check(lib().smc_set_waves_per_cu(self.h, int(w)))

    def set_specialization(self, mode: int):
        """SPECIALIZE_AUTO, SPECIALIZE_OFF or SPECIALIZE_REQUIRED."""
        self._check(lib().smc_set_specialization(self.h, int(mode)))

    def set_lanes_per_trajectory(self, lanes: int):
        """1, 2, 4, 8 or 16 lanes per trajectory (0: automatic)."""
        self._check(lib().smc_set_lanes_per_trajectory(self.h, int(lanes)))

    def set_kernel_occupancy(self, waves_per_simd: int):
        """Register budget of specialised kernels (0 = compiler default)."""
        self._check(lib().smc_set_kernel_occupancy(self.h, int(waves_per_simd)))

    def autotune(self, network, formula, p, pilot_n=1 << 16) -> dict:
        """Pick and apply the fastest launch configuration for this model's structure."""
        r = TuneResult()
        self._check(lib().smc_autotune(self.h, network.h, formula.h, ctypes.byref(p), int(pilot_n), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in TuneResult._fields_}

    def last_kernel(self) -> int:
        """KERNEL_GENERIC_SMALL, KERNEL_GENERIC or KERNEL_SPECIALIZED (-1: none yet)."""
        return int(lib().smc_last_kernel(self.h))

    def cus(self) -> int:
        return lib().smc_device_cus(self.h)

    def cancel(self):
        lib().smc_cancel(self.h)

    # -- handles ------------------------------------------------------------
    def network(self, net) -> "Network":
        return Network(self, net)

    def formula(self, network: "Network", text: str) -> "Formula":
        return Formula(self, network, text)

    # -- estimation ---------------------------------------------------------
    def estimate(self, network: "Network", formula: "Formula", p: Params) -> dict:
        r = Result()
        self._check(lib().smc_estimate(self.h, network.h, formula.h, ctypes.byref(p), ctypes.byref(r)))
        return r.as_dict()

    def estimate_batch(self, jobs) -> list:
        """jobs: list of (Network, Formula, Params).  last_call_seconds holds
        the wall time of the library call alone (without this marshalling)."""
        arr = (JobDesc * len(jobs))()
        for k, (n, f, p) in enumerate(jobs):
            arr[k].net = n.h
            arr[k].formula = f.h
            arr[k].params = p
        res = (Result * len(jobs))()
        t0 = time.perf_counter()
        rc = lib().smc_estimate_batch(self.h, arr, len(jobs), res)
        self.last_call_seconds = time.perf_counter() - t0
        self._check(rc)
        return [r.as_dict() for r in res]

    def autotune_batch(self, jobs, pilot_widen=1.0) -> dict:
        """smc_autotune_batch; jobs as for estimate_batch."""
        arr = (JobDesc * len(jobs))()
        for k, (n, f, p) in enumerate(jobs):
            arr[k].net = n.h
            arr[k].formula = f.h
            arr[k].params = p
        r = BatchTuneResult()
        self._check(lib().smc_autotune_batch(self.h, arr, len(jobs), float(pilot_widen), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in BatchTuneResult._fields_ if k != "pad_"}

    def estimate_batch_noalloc(self, jobs) -> list:
        """smc_estimate_batch_noalloc: at most NOALLOC_MAX_JOBS jobs, no allocation."""
        arr = (JobDesc * max(len(jobs), 1))()
        for k, (n, f, p) in enumerate(jobs):
            arr[k].net = n.h
            arr[k].formula = f.h
            arr[k].params = p
        res = (Result * max(len(jobs), 1))()
        self._check(lib().smc_estimate_batch_noalloc(self.h, arr, len(jobs), res))
        return [r.as_dict() for r in res[:len(jobs)]]

    def trajectories(self, network, formula, p: Params, first: int, count: int):
        ev = np.zeros(count, dtype=np.uint32)
        vr = np.zeros(count, dtype=np.uint8)
        self._check(lib().smc_trajectories(self.h, network.h, formula.h, ctypes.byref(p), first, count,
                                           ev.ctypes.data, vr.ctypes.data))
        return ev, vr & 1, vr >> 1

    def trajectories_device(self, network, formula, p: Params, first: int, count: int, events, verdict_reason):
        """smc_trajectories into device arrays (objects with data_ptr(), e.g.
        torch tensors of int32/uint8 on the context's device, or None)."""
        q = Params.from_buffer_copy(p)
        q.flags |= SMC_DEVICE_PTRS
        self._check(lib().smc_trajectories(self.h, network.h, formula.h, ctypes.byref(q), first, count,
                                           _dptr(events), _dptr(verdict_reason)))

    def wilson_next_device(self, successes, n, eps: float, z: float, paper_rounding=False):
        y = np.ascontiguousarray(successes, dtype=np.uint64)
        nn = np.ascontiguousarray(n, dtype=np.uint64)
        out = np.zeros(y.shape[0], dtype=np.uint64)
        self._check(lib().smc_wilson_next_device(
            self.h, _ptr(y, ctypes.c_uint64), _ptr(nn, ctypes.c_uint64), y.shape[0], eps, z,
            SMC_PAPER_ROUNDING if paper_rounding else 0, _ptr(out, ctypes.c_uint64)))
        return out

    def sample_state(self, network, p: Params, T: float, first: int, count: int):
        out = np.zeros((count, network.S), dtype=np.int32)
        self._check(lib().smc_sample_state(self.h, network.h, ctypes.byref(p), float(T), first, count,
                                           out.ctypes.data))
        return out

    def sample_state_device(self, network, p: Params, T: float, first: int, count: int, counts):
        """smc_sample_state into a device array (data_ptr(), int32 [count, S])."""
        q = Params.from_buffer_copy(p)
        q.flags |= SMC_DEVICE_PTRS
        self._check(lib().smc_sample_state(self.h, network.h, ctypes.byref(q), float(T), first, count,
                                           _dptr(counts)))


class Network:
    def __init__(self, ctx: Context, net):
        self.ctx = ctx
        self.S = int(np.asarray(net.x0).shape[0])
        self.M = int(np.asarray(net.rate).shape[0])
        x0 = np.ascontiguousarray(net.x0, dtype=np.int32)
        rate = np.ascontiguousarray(net.rate, dtype=np.float64)
        reac = np.ascontiguousarray(net.reactants, dtype=np.int32)
        ci = np.ascontiguousarray(net.chg_idx, dtype=np.int32)
        cv = np.ascontiguousarray(net.chg_val, dtype=np.int32)
        names = list(getattr(net, "names", [f"X{k}" for k in range(self.S)]))
        cnames = (ctypes.c_char_p * self.S)(*[n.encode() for n in names])
        d = NetDesc(self.S, self.M, _ptr(x0, ctypes.c_int32), _ptr(rate, ctypes.c_double),
                    _ptr(reac, ctypes.c_int32), _ptr(ci, ctypes.c_int32), _ptr(cv, ctypes.c_int32), cnames)
        out = ctypes.c_void_p()
        ctx._check(lib().smc_net_create(ctx.h, ctypes.byref(d), ctypes.byref(out)))
        self.h = out

    def set_rates(self, rate):
        r = np.ascontiguousarray(rate, dtype=np.float64)
        self.ctx._check(lib().smc_net_set_rates(self.h, _ptr(r, ctypes.c_double)))

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                lib().smc_net_destroy(self.h)
        except Exception:
            pass


class Formula:
    def __init__(self, ctx: Context, network: Network, text: str):
        self.ctx = ctx
        self.text = text
        out = ctypes.c_void_p()
        ctx._check(lib().smc_formula_compile(ctx.h, network.h, text.encode(), ctypes.byref(out)))
        self.h = out

    @property
    def horizon(self) -> float:
        return lib().smc_formula_horizon(self.h)

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                lib().smc_formula_destroy(self.h)
        except Exception:
            pass


# -- formula validation on the host (no device) ------------------------------
def formula_check(text: str, names):
    """(code, reason, horizon) of compiling `text` over species `names` for the
    GPU monitor, without a context: code is SMC_OK, SMC_E_PARSE,
    SMC_E_UNSUPPORTED or SMC_E_INVALID; horizon is None unless SMC_OK."""
    arr = (ctypes.c_char_p * max(len(names), 1))(*[n.encode() for n in names])
    hz = ctypes.c_double(math.nan)
    msg = ctypes.create_string_buffer(256)
    rc = lib().smc_formula_check(text.encode(), arr, len(names), ctypes.byref(hz), msg, 256)
    return rc, msg.value.decode(), (hz.value if rc == SMC_OK else None)


# -- Wilson formulas (host functions of the library) ------------------------
def z_value(confidence: float) -> float:
    return lib().smc_z_value(confidence)


def wilson_sample(p: float, eps: float, z: float) -> int:
    return int(lib().smc_wilson_sample(p, eps, z))


def wilson_sample_value(p: float, eps: float, z: float) -> float:
    return lib().smc_wilson_sample_value(p, eps, z)


def wilson_interval(k: int, n: int, z: float):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    lib().smc_wilson_interval(k, n, z, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def convex_hull(points) -> np.ndarray:
    """Facet planes (nx, ny, nz, d) of the convex hull of points [n, 3]."""
    pts = np.ascontiguousarray(points, dtype=np.float32)
    n = pts.shape[0]
    nf = lib().smc_convex_hull(_ptr(pts, ctypes.c_float), n, None, 0)
    out = np.zeros((max(nf, 0), 4), dtype=np.float32)
    if nf > 0:
        lib().smc_convex_hull(_ptr(pts, ctypes.c_float), n, _ptr(out, ctypes.c_float), nf)
    return out


class Surrogate:
    """MLP surrogate p(log10 rates) trained and evaluated by the library."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        out = ctypes.c_void_p()
        ctx._check(lib().smc_surrogate_create(ctx.h, seed, ctypes.byref(out)))
        self.h = out
        self.n_params = int(lib().smc_surrogate_param_count())

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        self.ctx._check(lib().smc_surrogate_get_params(self.h, _ptr(p, ctypes.c_float), self.n_params))
        return p

    def set_params(self, p):
        q = np.ascontiguousarray(p, dtype=np.float32)
        self.ctx._check(lib().smc_surrogate_set_params(self.h, _ptr(q, ctypes.c_float), q.size))

    def gradients(self, x, y, w=None):
        xx = np.ascontiguousarray(x, dtype=np.float32)
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ww = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        loss = ctypes.c_float()
        g = np.zeros(self.n_params - 6, dtype=np.float32)
        self.ctx._check(lib().smc_surrogate_gradients(
            self.h, _ptr(xx, ctypes.c_float), _ptr(yy, ctypes.c_float),
            None if ww is None else _ptr(ww, ctypes.c_float), xx.shape[0], ctypes.byref(loss),
            _ptr(g, ctypes.c_float)))
        return loss.value, g

    def train(self, x, y, w=None, steps=2000, lr=1e-3):
        xx = np.ascontiguousarray(x, dtype=np.float32)
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ww = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        losses = np.zeros(steps, dtype=np.float32)
        opts = TrainOpts(steps, lr, 0.0, 0.0, 0.0)
        self.ctx._check(lib().smc_surrogate_train(
            self.h, _ptr(xx, ctypes.c_float), _ptr(yy, ctypes.c_float),
            None if ww is None else _ptr(ww, ctypes.c_float), xx.shape[0], ctypes.byref(opts),
            _ptr(losses, ctypes.c_float)))
        return losses

    def query(self, x, threshold=0.5, margin=0.05):
        xx = np.ascontiguousarray(x, dtype=np.float32)
        n = xx.shape[0]
        p = np.zeros(n, dtype=np.float32)
        use = np.zeros(n, dtype=np.uint8)
        self.ctx._check(lib().smc_surrogate_query(self.h, xx.ctypes.data, n, threshold, margin, 0,
                                                  p.ctypes.data, use.ctypes.data))
        return p, use.astype(bool)

    def query_device(self, x, n: int, p_out, use_out=None, threshold=0.5, margin=0.05):
        """smc_surrogate_query on device arrays (data_ptr(): x float32 [n, 3],
        p_out float32 [n], use_out uint8 [n] or None)."""
        self.ctx._check(lib().smc_surrogate_query(self.h, _dptr(x), int(n), threshold, margin, SMC_DEVICE_PTRS,
                                                  _dptr(p_out), _dptr(use_out)))

    def calibrate(self, x, lo, hi, threshold=0.5, bound=0.01, min_margin=0.05):
        """Calibrate the gate on held-out estimates; returns (margin, share
        answered), margin -1 when the gate refuses every query."""
        xx = np.ascontiguousarray(x, dtype=np.float32)
        ll = np.ascontiguousarray(lo, dtype=np.float64)
        hh = np.ascontiguousarray(hi, dtype=np.float64)
        m, share = ctypes.c_float(), ctypes.c_float()
        self.ctx._check(lib().smc_surrogate_calibrate(self.h, xx.ctypes.data, ll.ctypes.data, hh.ctypes.data,
                                                      xx.shape[0], threshold, bound, min_margin,
                                                      ctypes.byref(m), ctypes.byref(share)))
        return m.value, share.value

    def confirm(self, p, use, successes, trials, threshold=0.5):
        """smc_surrogate_confirm on host arrays; returns the confirmed gate."""
        pp = np.ascontiguousarray(p, dtype=np.float32)
        uu = np.ascontiguousarray(use, dtype=np.uint8).copy()
        ss = np.ascontiguousarray(successes, dtype=np.uint64)
        tt = np.ascontiguousarray(trials, dtype=np.uint64)
        self.ctx._check(lib().smc_surrogate_confirm(self.h, pp.ctypes.data, ss.ctypes.data, tt.ctypes.data,
                                                    pp.shape[0], threshold, 0, uu.ctypes.data))
        return uu.astype(bool)

    def confirm_device(self, p, successes, trials, n: int, use, threshold=0.5):
        """smc_surrogate_confirm on device arrays (data_ptr(): p float32 [n],
        successes and trials 64-bit [n], use uint8 [n], updated in place)."""
        self.ctx._check(lib().smc_surrogate_confirm(self.h, _dptr(p), _dptr(successes), _dptr(trials), int(n),
                                                    threshold, SMC_DEVICE_PTRS, _dptr(use)))

    def neighbourhood(self) -> float:
        """The calibrated gate's neighbourhood size (log10 units; 0: none)."""
        return float(lib().smc_surrogate_neighbourhood(self.h))

    def hull(self) -> np.ndarray:
        nf = lib().smc_surrogate_hull(self.h, None, 0)
        out = np.zeros((max(nf, 0), 4), dtype=np.float32)
        if nf > 0:
            lib().smc_surrogate_hull(self.h, _ptr(out, ctypes.c_float), nf)
        return out

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                lib().smc_surrogate_destroy(self.h)
        except Exception:
            pass
