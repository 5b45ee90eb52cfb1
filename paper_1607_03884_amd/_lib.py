"""ctypes binding of librkchem.so (argument marshalling only).

Device memory and streams come from PyTorch tensors; every step of the
integration runs in the library's HIP kernels.  If the library is missing the
calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librkchem.so")

RK_OK = 0
STATUS_NAMES = {0: "ok", 1: "step_limit", 2: "h_underflow", 3: "nonfinite"}


class RkStats(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int64), ("steps", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("newton_iters", ctypes.c_int64), ("newton_fail", ctypes.c_int64),
                ("f_evals", ctypes.c_int64), ("jac_evals", ctypes.c_int64), ("lu_factor", ctypes.c_int64),
                ("n_failed", ctypes.c_int64), ("max_steps", ctypes.c_int32), ("min_steps", ctypes.c_int32),
                ("d_hist64", ctypes.c_int64 * 20), ("d_hist32", ctypes.c_int64 * 20),
                ("d_mean64", ctypes.c_double), ("d_mean32", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("fp32_fallback", ctypes.c_int64), ("nbins_used", ctypes.c_int32), ("grid_used", ctypes.c_int32),
                ("predictor_kept", ctypes.c_int64), ("predictor_fallback", ctypes.c_int64),
                ("d_hist64_queue", ctypes.c_int64 * 20), ("d_mean64_queue", ctypes.c_double),
                ("tile_used", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTS = ["mech_load", "mech_free", "mech_dims", "radau_integrate", "radau_integrate_noalloc", "stats_get",
           "radau_set_option",
           "rk_last_error", "rk_dbg_rhs", "rk_dbg_jacobian", "rk_dbg_lu_solve",
           "rk_mlp_create", "rk_mlp_free", "rk_mlp_param_count", "rk_mlp_set_params", "rk_mlp_get_params",
           "rk_mlp_forward", "rk_mlp_grads", "rk_mlp_train_step", "rk_mlp_last_error"]

_lib = None


class RkError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RkError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.mech_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.mech_free.argtypes = [vp]
        L.mech_free.restype = None
        L.mech_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.radau_integrate.argtypes = [vp, i64, dbl, vp, vp, dbl, dbl, vp]
        L.radau_integrate_noalloc.argtypes = [vp, i64, dbl, vp, vp, dbl, dbl, vp]
        L.stats_get.argtypes = [vp, ctypes.POINTER(RkStats), vp, vp]
        L.radau_set_option.argtypes = [vp, ctypes.c_char_p, ctypes.c_char_p]
        L.rk_last_error.restype = ctypes.c_char_p
        L.rk_dbg_rhs.argtypes = [vp, i64, vp, vp, vp]
        L.rk_dbg_jacobian.argtypes = [vp, i64, vp, vp, vp]
        L.rk_dbg_lu_solve.argtypes = [vp, i64, ctypes.c_int, dbl, vp, vp, vp, vp, vp]
        L.rk_mlp_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp)]
        L.rk_mlp_free.argtypes = [vp]
        L.rk_mlp_free.restype = None
        L.rk_mlp_param_count.argtypes = [vp]
        L.rk_mlp_param_count.restype = i64
        L.rk_mlp_set_params.argtypes = [vp, vp, i64]
        L.rk_mlp_get_params.argtypes = [vp, vp, i64]
        L.rk_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
        L.rk_mlp_grads.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.rk_mlp_train_step.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp]
        L.rk_mlp_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != RK_OK:
        raise RkError(f"{what} failed ({rc}): {lib().rk_last_error().decode()}")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _check_states(t, rows: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise RkError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.dim() != 2 or t.shape[0] != rows:
        raise RkError(f"{name} must have shape [{rows}, n] (component-major)")


class Mechanism:
    """A mechanism uploaded to the current device (owned library handle)."""

    def __init__(self, path: str):
        h = ctypes.c_void_p()
        _check(lib().mech_load(path.encode(), ctypes.byref(h)), "mech_load")
        self._h = h
        K, R = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mech_dims(h, ctypes.byref(K), ctypes.byref(R)), "mech_dims")
        self.K, self.R = K.value, R.value
        self.N = self.K + 1

    def close(self):
        if getattr(self, "_h", None):
            lib().mech_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: str, value) -> None:
        _check(lib().radau_set_option(self._h, key.encode(), str(value).encode()), f"radau_set_option({key})")

    def integrate(self, y_in, dt: float, atol: float = 1e-10, rtol: float = 1e-6, y_out=None, stream=None):
        """y_in: [K+2, n] float64 CUDA tensor (rows T, Y_1..Y_K, P).  Returns y_out."""
        import torch
        _check_states(y_in, self.K + 2, "y_in")
        n = y_in.shape[1]
        if y_out is None:
            y_out = torch.empty_like(y_in)
        _check_states(y_out, self.K + 2, "y_out")
        _check(lib().radau_integrate(self._h, n, float(dt), y_in.data_ptr(), y_out.data_ptr(), float(atol),
                                     float(rtol), _stream_ptr(stream)), "radau_integrate")
        return y_out

    def integrate_noalloc(self, y_in, dt: float, atol: float = 1e-10, rtol: float = 1e-6, y_out=None, stream=None):
        """As integrate, through radau_integrate_noalloc (the library allocates
        nothing; y_out must be given by callers that cannot allocate)."""
        import torch
        _check_states(y_in, self.K + 2, "y_in")
        n = y_in.shape[1]
        if y_out is None:
            y_out = torch.empty_like(y_in)
        _check_states(y_out, self.K + 2, "y_out")
        _check(lib().radau_integrate_noalloc(self._h, n, float(dt), y_in.data_ptr(), y_out.data_ptr(), float(atol),
                                             float(rtol), _stream_ptr(stream)), "radau_integrate_noalloc")
        return y_out

    def stats(self, per_state: bool = False) -> dict:
        s = RkStats()
        steps = status = None
        args = [None, None]
        if per_state:
            n = self._last_n()
            steps = np.zeros(n, dtype=np.int32)
            status = np.zeros(n, dtype=np.int32)
            args = [steps.ctypes.data, status.ctypes.data]
        _check(lib().stats_get(self._h, ctypes.byref(s), *args), "stats_get")
        out = {f: getattr(s, f) for f, _ in RkStats._fields_ if not f.startswith("d_hist")}
        out["d_hist64"] = list(s.d_hist64)
        out["d_hist32"] = list(s.d_hist32)
        out["d_hist64_queue"] = list(s.d_hist64_queue)
        if per_state:
            out["per_state_steps"] = steps
            out["per_state_status"] = status
        return out

    def _last_n(self) -> int:
        s = RkStats()
        _check(lib().stats_get(self._h, ctypes.byref(s), None, None), "stats_get")
        return int(s.n_states)

    def dbg_rhs(self, y, stream=None):
        import torch
        _check_states(y, self.K + 2, "y")
        f = torch.empty((self.N, y.shape[1]), dtype=torch.float64, device=y.device)
        _check(lib().rk_dbg_rhs(self._h, y.shape[1], y.data_ptr(), f.data_ptr(), _stream_ptr(stream)), "rk_dbg_rhs")
        return f

    def dbg_jacobian(self, y, stream=None):
        import torch
        _check_states(y, self.K + 2, "y")
        J = torch.empty((self.N * self.N, y.shape[1]), dtype=torch.float64, device=y.device)
        _check(lib().rk_dbg_jacobian(self._h, y.shape[1], y.data_ptr(), J.data_ptr(), _stream_ptr(stream)),
               "rk_dbg_jacobian")
        return J

    def dbg_lu_solve(self, J, b, h: float, fp32: bool = False, sc=None, stream=None):
        """x1 = E1^-1 b1, x2 + i x3 = E2^-1 (b2 + i b3) with the integrator's own
        factorisation (J: [N*N, n], b: [3*N, n], sc: [N, n] error weights)."""
        import torch
        n = J.shape[1]
        for t, rows, name in ((J, self.N * self.N, "J"), (b, 3 * self.N, "b")):
            if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (rows, n):
                raise RkError(f"{name} must be a contiguous float64 CUDA tensor of shape [{rows}, {n}]")
        if sc is None:
            sc = torch.ones((self.N, n), dtype=torch.float64, device=J.device)
        x = torch.empty_like(b)
        _check(lib().rk_dbg_lu_solve(self._h, n, int(bool(fp32)), float(h), J.data_ptr(), sc.data_ptr(),
                                     b.data_ptr(), x.data_ptr(), _stream_ptr(stream)), "rk_dbg_lu_solve")
        return x
