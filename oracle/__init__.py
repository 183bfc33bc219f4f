"""FP64 CPU oracle for PINS -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never calls it.

``oracle/pins_oracle.c`` is the plain sequential Alg. 2 / Alg. 1 in double
precision; it is built with gcc into ``oracle/liboracle.so`` and called
through ctypes here.  ``oracle.lp`` holds independent checks of LP optima
(permutation brute force, vertex enumeration, 1-D monotone coupling, scipy's
HiGHS) and the 2x2 closed form of the entropic plan.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pins_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        compile_to(_SRC, tmp)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("K", ctypes.c_int), ("T1", ctypes.c_int), ("T2", ctypes.c_int),
                ("warm_tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("final_tol", ctypes.c_double),
                ("cg_rtol", ctypes.c_double), ("cg_max", ctypes.c_int), ("ls_beta", ctypes.c_double),
                ("ls_c1", ctypes.c_double), ("ls_max", ctypes.c_int), ("rho", ctypes.c_double),
                ("budget", ctypes.c_double), ("rho_levels", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("eps", ctypes.c_double), ("resid", ctypes.c_double),
                ("dual", ctypes.c_double), ("gap", ctypes.c_double), ("entropy", ctypes.c_double),
                ("outer", ctypes.c_int), ("sinkhorn", ctypes.c_int), ("newton", ctypes.c_int),
                ("cg", ctypes.c_int), ("fallbacks", ctypes.c_int), ("flags", ctypes.c_int),
                ("nnz_last", ctypes.c_int), ("levels_last", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def compile_to(src: str, out: str) -> str:
    """Compile an oracle source file to a shared library at ``out``."""
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                           "-ffp-contract=off", "-I", _HERE, "-o", out, src, "-lm"])
    return out


def load(path: str):
    """Load an oracle shared library and declare its C signatures."""
    L = ctypes.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def _declare(L):
    D = ctypes.POINTER(ctypes.c_double)
    L.oracle_default_params.argtypes = [ctypes.POINTER(Params)]
    L.oracle_cost_points.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, D, D, ctypes.c_double, D]
    L.oracle_cost_grid.argtypes = [ctypes.c_int, ctypes.c_double, D]
    L.oracle_pins.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, ctypes.POINTER(Params), D, D, D,
                              ctypes.POINTER(Stats)]
    L.oracle_pins_trace.argtypes = L.oracle_pins.argtypes + [D]
    L.oracle_sinkhorn.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, D, D, D, ctypes.POINTER(Stats)]
    L.oracle_sinkhorn_row.argtypes = [ctypes.c_int, ctypes.c_int, D, D, ctypes.c_double, D, D, D]
    L.oracle_sinkhorn_col.argtypes = [ctypes.c_int, ctypes.c_int, D, D, ctypes.c_double, D, D]
    L.oracle_recover.argtypes = [ctypes.c_int, ctypes.c_int, D, ctypes.c_double, D, D, D]


def _p(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def default_params(**kw) -> Params:
    p = Params()
    lib().oracle_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def cost_points(x, y, scale=0.0):
    x, y = _f64(x), _f64(y)
    m, d = x.shape
    n = y.shape[0]
    C = np.empty((m, n))
    lib().oracle_cost_points(m, n, d, _p(x), _p(y), scale, _p(C))
    return C


def cost_grid(s, scale=0.0):
    C = np.empty((s * s, s * s))
    lib().oracle_cost_grid(s, scale, _p(C))
    return C


def pins(C, a, b, want_plan=True, trace=False, **kw):
    """Run Alg. 2 on dense C.  Returns dict(alpha, beta, X, status, [trace], **stats).

    trace rows (one per outer iteration): Sinkhorn sweeps, Newton steps, CG
    iterations, terminal residual, Sparsify level, <C, X^{k+1}>, nnz(S), fallbacks.
    """
    C, a, b = _f64(C), _f64(a), _f64(b)
    m, n = C.shape
    p = default_params(**kw)
    alpha = np.empty(m)
    beta = np.empty(n)
    X = np.empty((m, n)) if want_plan else None
    tr = np.zeros((p.K, 8)) if trace else None
    st = Stats()
    rc = lib().oracle_pins_trace(m, n, _p(C), _p(a), _p(b), ctypes.byref(p), _p(alpha), _p(beta),
                                 _p(X) if X is not None else None, ctypes.byref(st),
                                 _p(tr) if tr is not None else None)
    out = st.as_dict()
    out.update(alpha=alpha, beta=beta, X=X, status=rc)
    if trace:
        out["trace"] = tr
    return out


def sinkhorn(C, a, b, eps, tol=1e-14, maxit=200000, want_plan=True):
    """Alg. 1 at regularisation eps on C (standard-form potentials)."""
    C, a, b = _f64(C), _f64(a), _f64(b)
    m, n = C.shape
    alpha = np.empty(m)
    beta = np.empty(n)
    X = np.empty((m, n)) if want_plan else None
    st = Stats()
    rc = lib().oracle_sinkhorn(m, n, _p(C), _p(a), _p(b), eps, tol, maxit, _p(alpha), _p(beta),
                               _p(X) if X is not None else None, ctypes.byref(st))
    out = st.as_dict()
    out.update(alpha=alpha, beta=beta, X=X, status=rc)
    return out


def sinkhorn_row(Ck, a, eta, f, g):
    Ck, a, g = _f64(Ck), _f64(a), _f64(g)
    f = _f64(f).copy()
    m, n = Ck.shape
    err = ctypes.c_double(0.0)
    lib().oracle_sinkhorn_row(m, n, _p(Ck), _p(a), eta, _p(f), _p(g), ctypes.byref(err))
    return f, err.value


def sinkhorn_col(Ck, b, eta, f, g):
    Ck, b, f = _f64(Ck), _f64(b), _f64(f)
    g = _f64(g).copy()
    m, n = Ck.shape
    lib().oracle_sinkhorn_col(m, n, _p(Ck), _p(b), eta, _p(f), _p(g))
    return g


def recover(Ck, eta, f, g):
    Ck, f, g = _f64(Ck), _f64(f), _f64(g)
    m, n = Ck.shape
    X = np.empty((m, n))
    lib().oracle_recover(m, n, _p(Ck), eta, _p(f), _p(g), _p(X))
    return X
