"""CPU FP64 oracle (ctypes binding of liboracle.so).

TEST INFRASTRUCTURE ONLY: the independent reference for the HIP library.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg import
this package; the product path never does.  It shares no code with the HIP
library: its own parser, thermochemistry, Jacobian, LU and Radau IIA.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["mech.c", "chem.c", "radau.c", "ros.c"]

OK, STEP_LIMIT, H_UNDERFLOW, NONFINITE = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, -ffp-contract=off, OpenMP)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    deps = srcs + [os.path.join(HERE, "oracle.h"), os.path.join(HERE, "chem_generic.inc")]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


class Opts(ctypes.Structure):
    _fields_ = [("kmax", ctypes.c_int), ("kappa", ctypes.c_double), ("h0", ctypes.c_double),
                ("nmax", ctypes.c_int), ("untransformed", ctypes.c_int), ("isothermal", ctypes.c_int),
                ("fd_jac", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nstep", ctypes.c_int32), ("naccept", ctypes.c_int32),
                ("nreject", ctypes.c_int32), ("nnewton", ctypes.c_int32), ("nnewtfail", ctypes.c_int32),
                ("nfev", ctypes.c_int32), ("njev", ctypes.c_int32), ("nlu", ctypes.c_int32),
                ("warm", ctypes.c_int32), ("h_first", ctypes.c_double)]


RESULT_DTYPE = np.dtype([(n, np.int32) for n in ("status", "nstep", "naccept", "nreject", "nnewton",
                                                 "nnewtfail", "nfev", "njev", "nlu", "warm")] +
                        [("h_first", np.float64)],
                        align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_mech_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
        L.or_mech_free.argtypes = [ctypes.c_void_p]
        L.or_mech_dims.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 3
        L.or_thermo.argtypes = [ctypes.c_void_p, ctypes.c_double, dp, dp, dp]
        L.or_rates.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp, dp]
        L.or_rates2.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp, dp, dp, dp]
        L.or_rhs.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_rhs_iso.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_jac.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_jac_iso.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_jac_cs.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_jac_fd.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, dp]
        L.or_integrate_rodas3.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, dp, dp, ctypes.c_double,
                                          ctypes.c_double, ctypes.POINTER(Opts), ctypes.c_void_p, ctypes.c_int]
        L.or_rodas3_fixed_steps.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int, dp]
        L.or_rodas3_linear_step.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.or_rodas3_table.argtypes = [dp, dp, dp, dp, dp]
        L.or_jac_fd_quadratic.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.or_radau_constants.argtypes = [dp] * 7
        L.or_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.or_integrate_batch.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, dp, dp,
                                         ctypes.c_double, ctypes.c_double, ctypes.POINTER(Opts), dp,
                                         ctypes.c_void_p, ctypes.c_int]
        L.or_integrate_batch2.argtypes = L.or_integrate_batch.argtypes + [dp]
        L.or_integrate_batch3.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, dp, dp,
                                          ctypes.c_double, ctypes.c_double, ctypes.POINTER(Opts), dp, dp,
                                          ctypes.c_void_p, ctypes.c_int, dp]
        L.or_integrate_linear.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(Opts), dp, ctypes.POINTER(Result), dp, ctypes.c_int]
        L.or_fixed_steps.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().or_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Mech:
    """A mechanism loaded by the oracle's own reader."""

    def __init__(self, path: str):
        h = ctypes.c_void_p()
        rc = lib().or_mech_load(path.encode(), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle could not read mechanism {path} (rc={rc})")
        self.h = h
        K, R, E = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib().or_mech_dims(h, ctypes.byref(K), ctypes.byref(R), ctypes.byref(E))
        self.K, self.R, self.E = K.value, R.value, E.value
        self.N = self.K + 1

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_mech_free(self.h)
            self.h = None

    # -- single-state evaluations ------------------------------------------------
    def thermo(self, T: float):
        cp, h, s = (np.zeros(self.K) for _ in range(3))
        lib().or_thermo(self.h, T, _p(cp), _p(h), _p(s))
        return cp, h, s

    def rates(self, y: np.ndarray, P: float):
        y = np.ascontiguousarray(y, dtype=np.float64)
        q, w = np.zeros(self.R), np.zeros(self.K)
        lib().or_rates(self.h, _p(y), P, _p(q), _p(w))
        return q, w

    def rates_fr(self, y: np.ndarray, P: float):
        """(q, wdot, forward part, reverse part) with q = qf - qr."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        q, w, qf, qr = np.zeros(self.R), np.zeros(self.K), np.zeros(self.R), np.zeros(self.R)
        lib().or_rates2(self.h, _p(y), P, _p(q), _p(w), _p(qf), _p(qr))
        return q, w, qf, qr

    def rhs(self, y: np.ndarray, P: float, isothermal: bool = False) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.N)
        (lib().or_rhs_iso if isothermal else lib().or_rhs)(self.h, _p(y), P, _p(f))
        return f

    def jac(self, y: np.ndarray, P: float, isothermal: bool = False) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros((self.N, self.N))
        (lib().or_jac_iso if isothermal else lib().or_jac)(self.h, _p(y), P, _p(J))
        return J

    def jac_fd(self, y: np.ndarray, P: float, h: float, atol: float = 1e-10, rtol: float = 1e-6) -> np.ndarray:
        """First-order forward-difference Jacobian (CVODE-style increments)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        f0 = self.rhs(y, P)
        J = np.zeros((self.N, self.N))
        lib().or_jac_fd(self.h, _p(y), P, _p(f0), h, atol, rtol, _p(J))
        return J

    def jac_cs(self, y: np.ndarray, P: float) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros((self.N, self.N))
        lib().or_jac_cs(self.h, _p(y), P, _p(J))
        return J

    # -- integration ----------------------------------------------------------------
    def integrate(self, states: np.ndarray, dt: float, atol: float = 1e-10, rtol: float = 1e-6,
                  opts: Optional[Opts] = None, h0: Optional[np.ndarray] = None, nthreads: int = 0):
        """states: [n, K+2] rows (T, Y, P).  Returns (out rows, per-state results)."""
        st = np.ascontiguousarray(states, dtype=np.float64)
        n = st.shape[0]
        assert st.shape[1] == self.K + 2
        out = np.zeros_like(st)
        res = np.zeros(n, dtype=RESULT_DTYPE)
        o = opts or default_opts()
        h0p = _p(np.ascontiguousarray(h0, dtype=np.float64)) if h0 is not None else None
        if h0 is not None:
            h0 = np.ascontiguousarray(h0, dtype=np.float64)
            h0p = _p(h0)
        lib().or_integrate_batch(self.h, n, dt, _p(st), _p(out), atol, rtol, ctypes.byref(o), h0p,
                                 res.ctypes.data_as(ctypes.c_void_p), nthreads)
        return out, res

    def integrate_rodas3(self, states: np.ndarray, dt: float, atol: float = 1e-10, rtol: float = 1e-6,
                         opts: Optional[Opts] = None, nthreads: int = 0):
        """Rodas3 (Rosenbrock) over [0, dt]; as integrate."""
        st = np.ascontiguousarray(states, dtype=np.float64)
        n = st.shape[0]
        assert st.shape[1] == self.K + 2
        out = np.zeros_like(st)
        res = np.zeros(n, dtype=RESULT_DTYPE)
        o = opts or default_opts()
        lib().or_integrate_rodas3(self.h, n, dt, _p(st), _p(out), atol, rtol, ctypes.byref(o),
                                  res.ctypes.data_as(ctypes.c_void_p), nthreads)
        return out, res

    def rodas3_fixed_steps(self, state: np.ndarray, dt: float, nsteps: int) -> np.ndarray:
        st = np.ascontiguousarray(state, dtype=np.float64)
        out = np.zeros(self.N)
        lib().or_rodas3_fixed_steps(self.h, _p(st), dt, nsteps, _p(out))
        return out

    def integrate_warm(self, states: np.ndarray, dt: float, hw: Optional[np.ndarray], zw: Optional[np.ndarray],
                       atol: float = 1e-10, rtol: float = 1e-6, opts: Optional[Opts] = None, nthreads: int = 0):
        """Integration with a per-state warm start for the first step attempt:
        step size hw [n] (<= 0 or None: the default rule) and Newton starting
        values zw [n, 3, N] (None: zero); a warm attempt whose Newton iteration
        does not converge restarts the state cold.  res["warm"]: 1 kept,
        2 restarted cold."""
        st = np.ascontiguousarray(states, dtype=np.float64)
        n = st.shape[0]
        out = np.zeros_like(st)
        res = np.zeros(n, dtype=RESULT_DTYPE)
        o = opts or default_opts()
        hwp = zwp = None
        if hw is not None:
            hw = np.ascontiguousarray(hw, dtype=np.float64)
            assert hw.shape == (n,)
            hwp = _p(hw)
        if zw is not None:
            zw = np.ascontiguousarray(zw, dtype=np.float64)
            assert zw.shape == (n, 3, self.N)
            zwp = _p(zw)
        lib().or_integrate_batch3(self.h, n, dt, _p(st), _p(out), atol, rtol, ctypes.byref(o), hwp, zwp,
                                  res.ctypes.data_as(ctypes.c_void_p), nthreads, None)
        return out, res

    def integrate_first_step(self, states: np.ndarray, dt: float, atol: float = 1e-10, rtol: float = 1e-6,
                             nthreads: int = 0):
        """As integrate, also returning the first accepted step's stage
        increments Z [n, 3, N] (zeros for states that never accepted a step)."""
        st = np.ascontiguousarray(states, dtype=np.float64)
        n = st.shape[0]
        out = np.zeros_like(st)
        res = np.zeros(n, dtype=RESULT_DTYPE)
        z = np.zeros((n, 3, self.N))
        o = default_opts()
        lib().or_integrate_batch2(self.h, n, dt, _p(st), _p(out), atol, rtol, ctypes.byref(o), None,
                                  res.ctypes.data_as(ctypes.c_void_p), nthreads, _p(z))
        return out, res, z

    def fixed_steps(self, state: np.ndarray, dt: float, nsteps: int) -> np.ndarray:
        st = np.ascontiguousarray(state, dtype=np.float64)
        out = np.zeros_like(st)
        lib().or_fixed_steps(self.h, _p(st), dt, nsteps, _p(out))
        return out


def radau_constants():
    A, T, Ti = np.zeros(9), np.zeros(9), np.zeros(9)
    c, b, ev, d = np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3)
    lib().or_radau_constants(_p(A), _p(c), _p(b), _p(ev), _p(T), _p(Ti), _p(d))
    return dict(A=A.reshape(3, 3), c=c, b=b, gamma=ev[0], alpha=ev[1], beta=ev[2],
                T=T.reshape(3, 3), Tinv=Ti.reshape(3, 3), d=d)


def integrate_linear(M: np.ndarray, y0: np.ndarray, dt: float, atol: float, rtol: float,
                     opts: Optional[Opts] = None, cap: int = 100000):
    M = np.ascontiguousarray(M, dtype=np.float64)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    N = y0.shape[0]
    out = np.zeros(N)
    res = Result()
    hrec = np.zeros(cap)
    o = opts or default_opts()
    lib().or_integrate_linear(N, _p(M), _p(y0), dt, atol, rtol, ctypes.byref(o), _p(out), ctypes.byref(res),
                              _p(hrec), cap)
    return out, res, hrec[:min(res.naccept, cap)].copy()


def jac_fd_quadratic(A: np.ndarray, y: np.ndarray, h: float, atol: float, rtol: float) -> np.ndarray:
    """The oracle's forward-difference Jacobian of f_i(y) = sum_j A_ij y_j^2."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = y.shape[0]
    J = np.zeros((N, N))
    lib().or_jac_fd_quadratic(N, _p(A), _p(y), h, atol, rtol, _p(J))
    return J


def rodas3_table():
    g = np.zeros(1)
    a, c = np.zeros(16), np.zeros(16)
    m, e = np.zeros(4), np.zeros(4)
    lib().or_rodas3_table(_p(g), _p(a), _p(c), _p(m), _p(e))
    return dict(gamma=float(g[0]), a=a.reshape(4, 4), c=c.reshape(4, 4), m=m, e=e)


def rodas3_linear_step(M: np.ndarray, y0: np.ndarray, h: float) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float64)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    y1 = np.zeros_like(y0)
    lib().or_rodas3_linear_step(len(y0), _p(M), _p(y0), h, _p(y1))
    return y1
