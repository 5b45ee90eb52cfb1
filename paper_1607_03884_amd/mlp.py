"""ctypes binding of the predictor network kernels (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np

from . import _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise _lib.RkError(f"{what} failed ({rc}): {_lib.lib().rk_mlp_last_error().decode()}")


def _stream(stream):
    import torch
    return (stream or torch.cuda.current_stream()).cuda_stream


class Mlp:
    """GELU multilayer perceptron on the current device (BF16 weights in every
    product, FP32 accumulation, FP32 master parameters, Adam)."""

    def __init__(self, dims: Sequence[int]):
        L = _lib.lib()
        arr = (ctypes.c_int32 * len(dims))(*dims)
        h = ctypes.c_void_p()
        _check(L.rk_mlp_create(len(dims), arr, ctypes.byref(h)), "rk_mlp_create")
        self._h = h
        self.dims = list(dims)
        self.count = int(L.rk_mlp_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().rk_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p: np.ndarray) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.lib().rk_mlp_set_params(self._h, p.ctypes.data, p.size), "rk_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.count, dtype=np.float32)
        _check(_lib.lib().rk_mlp_get_params(self._h, p.ctypes.data, p.size), "rk_mlp_get_params")
        return p

    def forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        _check(_lib.lib().rk_mlp_forward(self._h, x.shape[0], x.data_ptr(), y.data_ptr(), _stream(stream)),
               "rk_mlp_forward")
        return y

    def grads(self, x, t, mask, wout, stream=None):
        import torch
        g = torch.empty(self.count, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(_lib.lib().rk_mlp_grads(self._h, x.shape[0], x.data_ptr(), t.data_ptr(), mask.data_ptr(),
                                       wout.data_ptr(), g.data_ptr(), loss.data_ptr(), _stream(stream)), "rk_mlp_grads")
        return loss, g

    def train_step(self, x, t, mask, wout, inv_count: float, lr: float, loss_out, stream=None):
        _check(_lib.lib().rk_mlp_train_step(self._h, x.shape[0], x.data_ptr(), t.data_ptr(), mask.data_ptr(),
                                            wout.data_ptr(), float(inv_count), float(lr), loss_out.data_ptr(),
                                            _stream(stream)), "rk_mlp_train_step")


def init_params(dims: Sequence[int], seed: int) -> np.ndarray:
    """He-style seeded initialisation in the flat layout (W then b per layer)."""
    rng = np.random.default_rng(seed)
    parts = []
    for din, dout in zip(dims[:-1], dims[1:]):
        parts.append((rng.standard_normal((dout, din)) * np.sqrt(2.0 / din)).ravel())
        parts.append(np.zeros(dout))
    return np.concatenate(parts).astype(np.float32)
