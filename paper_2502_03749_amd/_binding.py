"""ctypes binding of libpins.so (include/pins.h) -- argument marshalling only.

Every step of the solve runs in the HIP library; nothing here computes any
part of the method.  If the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpins.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pins.h")

PINS_OK = 0
PINS_NOT_CONVERGED = 1
PINS_EINVAL = -1
PINS_ENOMEM = -2
PINS_EDEVICE = -3
PINS_ENUMERIC = -4
PINS_EUNSUPPORTED = -5

COST_DENSE, COST_POINTS, COST_GRID = 0, 1, 2
FP64, MIXED, MIXED_FAST = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20
SHIFT_IMPLICIT, SHIFT_MATERIALIZED = 0, 1
NKERN = 16
KERNEL_NAMES = ["row_lse", "col_lse", "col_merge", "grad", "grad_merge", "fill", "pcg_rows", "pcg", "ls", "update",
                "shift", "final", "setup", "pcg_wide"]

_D = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("max_outer", ctypes.c_int32), ("max_sinkhorn", ctypes.c_int32),
                ("max_newton", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32), ("warm_tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("final_tol", ctypes.c_double), ("cg_rtol", ctypes.c_double),
                ("ls_beta", ctypes.c_double), ("ls_c1", ctypes.c_double), ("ls_max", ctypes.c_int32),
                ("rho_levels", ctypes.c_int32), ("rho", ctypes.c_double), ("budget", ctypes.c_double),
                ("precision", ctypes.c_int32), ("shift_mode", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("profile_mask", ctypes.c_int32), ("hvp", ctypes.c_int32),
                ("hvp_switch", ctypes.c_int32), ("graphs", ctypes.c_int32), ("tile_rows", ctypes.c_int32 * 4)]


class TuneTrial(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("graphs", ctypes.c_int32), ("tile_rows", ctypes.c_int32 * 4),
                ("ms", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("d", ctypes.c_int32),
                ("grid_s", ctypes.c_int32), ("reserved", ctypes.c_int32), ("C", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("cost_scale", ctypes.c_double),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("cost", ctypes.c_double), ("eps", ctypes.c_double), ("resid", ctypes.c_double),
                ("dual", ctypes.c_double), ("gap", ctypes.c_double), ("entropy", ctypes.c_double),
                ("cost_scale", ctypes.c_double), ("time_ms", ctypes.c_double), ("status", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("sinkhorn_iters", ctypes.c_int32),
                ("newton_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("nnz_last", ctypes.c_int32), ("kern_ms", ctypes.c_double * NKERN),
                ("kern_calls", ctypes.c_int32 * NKERN), ("kern_work", ctypes.c_double * NKERN),
                ("group", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def scalars(self) -> dict:
        out = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("alpha", "beta", "X", "kern_ms",
                                                                            "kern_calls", "kern_work")}
        out["kern_ms"] = {KERNEL_NAMES[i]: self.kern_ms[i] for i in range(len(KERNEL_NAMES))}
        out["kern_calls"] = {KERNEL_NAMES[i]: self.kern_calls[i] for i in range(len(KERNEL_NAMES))}
        out["kern_work"] = {KERNEL_NAMES[i]: self.kern_work[i] for i in range(len(KERNEL_NAMES))}
        return out


class State(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("outer_done", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("F", _D), ("G", _D), ("A", _D), ("B", _D)]


class PinsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pins error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libpins.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpins.so is not built (run __graft_entry__.build() or "
                              "python paper_2502_03749_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.pins_abi_version.restype = ctypes.c_int
        L.pins_params_default.argtypes = [ctypes.POINTER(Params)]
        L.pins_params_default.restype = None
        L.pins_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.pins_destroy.argtypes = [vp]
        L.pins_destroy.restype = None
        L.pins_last_error.argtypes = [vp]
        L.pins_last_error.restype = ctypes.c_char_p
        L.pins_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Params),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.pins_solve.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(Result)]
        L.pins_solve_device.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(Result),
                                        vp]
        L.pins_solve_device_noalloc.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                                ctypes.POINTER(Result), vp]
        L.pins_solve_resume.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(State),
                                        ctypes.c_int32, ctypes.POINTER(State), ctypes.POINTER(Result)]
        L.pins_tune_batch_device.argtypes = [vp, ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Params),
                                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(Result), vp,
                                             ctypes.POINTER(Params), ctypes.POINTER(TuneTrial), ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int32)]
        L.pins_probe_exp_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D]
        L.pins_probe_texp.argtypes = [vp, vp, ctypes.c_int, vp]
        L.pins_solve_batch_device.argtypes = [vp, ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Params),
                                              ctypes.POINTER(Result), vp]
        L.pins_server_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                         ctypes.POINTER(Params), ctypes.POINTER(vp)]
        L.pins_server_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_int64)]
        L.pins_server_wait.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_double)]
        L.pins_server_last_error.argtypes = [vp]
        L.pins_server_last_error.restype = ctypes.c_char_p
        L.pins_server_destroy.argtypes = [vp]
        L.pins_server_destroy.restype = None
        _lib = L
    return _lib


def declared_functions() -> list:
    """Names of the functions include/pins.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pins_[a-z_]+)\s*\(", txt)))


def params(**kw) -> Params:
    p = Params()
    lib().pins_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "tile_rows":
            v = (ctypes.c_int32 * 4)(*v)
        setattr(p, k, v)
    return p


class Context:
    """A library context on one HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib().pins_create(device, ctypes.byref(h))
        if rc != PINS_OK:
            raise PinsError(rc, "pins_create(%d) failed" % device)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pins_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().pins_last_error(self.h).decode()

    def _check(self, rc):
        if rc < 0:
            raise PinsError(rc, self.last_error())
        return rc

    # -------------------------------------------------------------- host API
    def solve(self, kind, a, b, prm: Params, C=None, x=None, y=None, grid_s=0, cost_scale=0.0, want_plan=False):
        """pins_solve with numpy host arrays.  Returns dict(alpha, beta, X, **scalars)."""
        P, keep = _host_problem(kind, a, b, C, x, y, grid_s, cost_scale)
        R, outs = _host_result(P.m, P.n, want_plan)
        rc = self._check(lib().pins_solve(self.h, ctypes.byref(P), ctypes.byref(prm), ctypes.byref(R)))
        out = R.scalars()
        out.update(outs, rc=rc)
        return out

    def solve_resume(self, kind, a, b, prm: Params, state=None, stop=0, C=None, x=None, y=None, grid_s=0,
                     cost_scale=0.0, want_plan=False):
        """pins_solve_resume with numpy host arrays.

        state: None (start) or a dict(outer_done, flags, F, G, A, B) returned by an earlier call;
        stop: outer iterations completed when the call returns (0 = max_outer).
        Returns dict(alpha, beta, X, state, **scalars), state being the resume point reached.
        """
        P, keep = _host_problem(kind, a, b, C, x, y, grid_s, cost_scale)
        R, outs = _host_result(P.m, P.n, want_plan)
        m, n = P.m, P.n
        save = {k: np.empty(m if k in ("F", "A") else n) for k in ("F", "G", "A", "B")}
        S_out = State(**{k: v.ctypes.data_as(_D) for k, v in save.items()})
        S_in = None
        if state is not None:
            arr = {k: np.ascontiguousarray(state[k], np.float64) for k in ("F", "G", "A", "B")}
            keep.append(arr)
            S_in = State(m=arr["F"].size, n=arr["G"].size, outer_done=state["outer_done"],
                         flags=state.get("flags", 0), **{k: v.ctypes.data_as(_D) for k, v in arr.items()})
        rc = self._check(lib().pins_solve_resume(self.h, ctypes.byref(P), ctypes.byref(prm),
                                                 ctypes.byref(S_in) if S_in is not None else None, int(stop),
                                                 ctypes.byref(S_out), ctypes.byref(R)))
        out = R.scalars()
        out.update(outs, rc=rc, state=dict(save, outer_done=S_out.outer_done, flags=S_out.flags))
        return out

    # ------------------------------------------------------------ device API
    def solve_batch_device(self, problems, prm: Params, outs, stream=None):
        """pins_solve_batch_device.

        problems: list of dicts with kind, a, b and C | (x, y) | grid_s (torch CUDA float64 tensors or
        raw device pointers as ints); outs: list of dicts with alpha, beta and optional X (device).
        Returns (rc, [scalars per instance]).
        """
        P, R = self._batch_args(problems, outs)
        cnt = len(problems)
        rc = self._check(lib().pins_solve_batch_device(self.h, P, cnt, ctypes.byref(prm), R,
                                                       ctypes.c_void_p(stream or 0)))
        return rc, [R[q].scalars() for q in range(cnt)]

    @staticmethod
    def _batch_args(problems, outs):
        """Problem and Result arrays over device tensors (or raw device pointers)."""
        cnt = len(problems)
        P = (Problem * cnt)()
        R = (Result * cnt)()
        for q, pr in enumerate(problems):
            P[q].kind = pr["kind"]
            P[q].m = pr["m"]
            P[q].n = pr["n"]
            P[q].d = pr.get("d", 0)
            P[q].grid_s = pr.get("grid_s", 0)
            P[q].cost_scale = pr.get("cost_scale", 0.0)
            for f in ("C", "x", "y", "a", "b"):
                if pr.get(f) is not None:
                    setattr(P[q], f, _ptr(pr[f]))
            R[q].alpha = _ptr(outs[q]["alpha"])
            R[q].beta = _ptr(outs[q]["beta"])
            if outs[q].get("X") is not None:
                R[q].X = _ptr(outs[q]["X"])
        return P, R

    def tune_batch_device(self, problems, prm: Params, outs, max_lanes=4, reps=2, stream=None):
        """pins_tune_batch_device: the fastest lanes / graph replay / rows per tile for this batch.

        Same arguments as solve_batch_device.  Returns (best Params, [trials as dicts in order]).
        """
        P, R = self._batch_args(problems, outs)
        best = Params()
        maxt = 16
        trials = (TuneTrial * maxt)()
        nt = ctypes.c_int32(0)
        self._check(lib().pins_tune_batch_device(self.h, P, len(problems), ctypes.byref(prm), max_lanes, reps, R,
                                                 ctypes.c_void_p(stream or 0), ctypes.byref(best), trials, maxt,
                                                 ctypes.byref(nt)))
        out = [dict(streams=t.streams, graphs=t.graphs, tile_rows=list(t.tile_rows), ms=t.ms)
               for t in trials[:min(nt.value, maxt)]]
        return best, out

    def solve_device(self, problem, prm: Params, out, stream=None):
        cnt_rc, res = self.solve_batch_device([problem], prm, [out], stream)
        return cnt_rc, res[0]

    def solve_device_noalloc(self, problem, prm: Params, out, stream=None):
        """pins_solve_device_noalloc: pins_solve_device on the library's fixed device scratch."""
        P, R = self._batch_args([problem], [out])
        rc = self._check(lib().pins_solve_device_noalloc(self.h, P, ctypes.byref(prm), R,
                                                         ctypes.c_void_p(stream or 0)))
        return rc, R[0].scalars()


class Server:
    """pins_server: continuous admission of host-side requests onto concurrent
    batched solves (workers threads, each with its own context and stream)."""

    def __init__(self, prm: Params, device: int = 0, workers: int = 2, max_batch: int = 64, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        self._prm = prm
        rc = lib().pins_server_create(device, workers, max_batch, hbm_budget, ctypes.byref(prm), ctypes.byref(h))
        if rc != PINS_OK:
            raise PinsError(rc, "pins_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, kind, a, b, C=None, x=None, y=None, grid_s=0, cost_scale=0.0) -> int:
        a = np.ascontiguousarray(a, np.float64)
        b = np.ascontiguousarray(b, np.float64)
        P = Problem(kind=kind, m=a.size, n=b.size, d=0, grid_s=grid_s, cost_scale=cost_scale, a=a.ctypes.data,
                    b=b.ctypes.data)
        keep = [a, b]
        if C is not None:
            C = np.ascontiguousarray(C, np.float64)
            keep.append(C)
            P.C = C.ctypes.data
        if x is not None:
            x = np.ascontiguousarray(x, np.float64)
            y = np.ascontiguousarray(y, np.float64)
            keep += [x, y]
            P.x, P.y, P.d = x.ctypes.data, y.ctypes.data, x.shape[1]
        t = ctypes.c_int64(0)
        rc = lib().pins_server_submit(self.h, ctypes.byref(P), ctypes.byref(t))
        if rc != PINS_OK:
            raise PinsError(rc, "pins_server_submit failed")
        self._keep[t.value] = (a.size, b.size)
        return t.value

    def wait(self, ticket: int) -> dict:
        m, n = self._keep.pop(ticket)
        alpha, beta = np.empty(m), np.empty(n)
        R = Result(alpha=alpha.ctypes.data, beta=beta.ctypes.data)
        lat = ctypes.c_double(0.0)
        rc = lib().pins_server_wait(self.h, ticket, ctypes.byref(R), ctypes.byref(lat))
        if rc < 0:
            raise PinsError(rc, lib().pins_server_last_error(self.h).decode())
        out = R.scalars()
        out.update(alpha=alpha, beta=beta, rc=rc, latency_ms=lat.value)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().pins_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_problem(kind, a, b, C, x, y, grid_s, cost_scale):
    """A Problem over numpy host arrays, and the arrays it points into."""
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    keep = [a, b]
    P = Problem(kind=kind, m=a.size, n=b.size, d=0, grid_s=grid_s, cost_scale=cost_scale,
                a=a.ctypes.data, b=b.ctypes.data)
    if C is not None:
        C = np.ascontiguousarray(C, np.float64)
        keep.append(C)
        P.C = C.ctypes.data
    if x is not None:
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        keep += [x, y]
        P.x, P.y, P.d = x.ctypes.data, y.ctypes.data, x.shape[1]
    return P, keep


def _host_result(m, n, want_plan):
    """A Result with host output arrays alpha (m), beta (n) and optionally X (m x n)."""
    outs = dict(alpha=np.empty(m), beta=np.empty(n), X=np.empty((m, n)) if want_plan else None)
    R = Result(alpha=outs["alpha"].ctypes.data, beta=outs["beta"].ctypes.data,
               X=outs["X"].ctypes.data if want_plan else None)
    return R, outs


def _ptr(t):
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("device arrays must be contiguous")
        import torch

        if t.dtype != torch.float64:
            raise TypeError("device arrays must be float64")
        return t.data_ptr()
    raise TypeError("unsupported array type %r" % type(t))


def probe_exp_rate(device: int = 0, blocks: int = 8192, iters: int = 4096):
    """pins_probe_exp_rate: (float exponentials per second, kernel ms)."""
    rate, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().pins_probe_exp_rate(device, blocks, iters, ctypes.byref(rate), ctypes.byref(ms))
    if rc != PINS_OK:
        raise PinsError(rc, "pins_probe_exp_rate failed")
    return rate.value, ms.value


def probe_texp(x, y, stream=None):
    """pins_probe_texp: y = the FP64 dense passes' exp of x (float64 device tensors of equal size)."""
    if x.numel() != y.numel():
        raise ValueError("x and y must have the same size")
    rc = lib().pins_probe_texp(_ptr(x), _ptr(y), x.numel(), ctypes.c_void_p(stream or 0))
    if rc != PINS_OK:
        raise PinsError(rc, "pins_probe_texp failed")


def workspace_bytes(problems, prm: Params) -> int:
    cnt = len(problems)
    P = (Problem * cnt)()
    for q, pr in enumerate(problems):
        P[q].kind = pr["kind"]
        P[q].m = pr["m"]
        P[q].n = pr["n"]
        P[q].d = pr.get("d", 0)
        P[q].grid_s = pr.get("grid_s", 0)
        P[q].a = 1
        P[q].b = 1
        P[q].C = 1
        P[q].x = 1
        P[q].y = 1
    out = ctypes.c_size_t(0)
    rc = lib().pins_workspace_bytes(P, cnt, ctypes.byref(prm), ctypes.byref(out))
    if rc != PINS_OK:
        raise PinsError(rc, "pins_workspace_bytes failed")
    return out.value
