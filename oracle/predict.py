"""Warm-start values of the learned first-step predictor, computed on the CPU
(test infrastructure only: tests and the CPU baseline use it, the library
does not).

A predictor file holds the network widths, the input/output standardisation
and the FP32 parameters of an MLP (see oracle/mlp.py for the network).  For a
state (T, Y, P) the input is [T / 1000, ln(P / 1 atm), Y_1..Y_K], standardised
and rounded to FP32.  The outputs, de-standardised to t, decode as
  * stage values z_ic = sign(t) (e^|t| - 1) sc_c, sc_c = atol + rtol |y0_c|,
    with t clipped to [-40, 40]   (t is symlog(z / sc));
  * first step size h = dt 2^-q, q = round(-log2(10) t), t clipped to
    [-15, 0]                      (t is log10(h / dt));
  * predicted step attempts 10^t, t clipped to [0, 7];
and a non-finite output decodes to 0 (for h: the default initial step).
"""
from __future__ import annotations

import numpy as np

from .mlp import MlpRef

P_ATM = 101325.0


def load(path: str) -> dict:
    """Parse a predictor file (whitespace-separated tokens)."""
    with open(path) as fh:
        tok = fh.read().split()
    pos = 0

    def take(n=1):
        nonlocal pos
        out = tok[pos:pos + n]
        pos += n
        return out

    def word(w):
        got = take()[0]
        if got != w:
            raise ValueError(f"predictor file: expected {w!r}, found {got!r}")

    word("rkpred")
    if take()[0] != "1":
        raise ValueError("predictor file: unsupported version")
    word("mech")
    name = take()[0]
    word("K")
    K = int(take()[0])
    word("dt")
    dt = float(take()[0])
    word("dims")
    L = int(take()[0])
    dims = [int(v) for v in take(L)]
    out = dict(mech=name, K=K, dt=dt, dims=dims)
    for key, cnt in (("in_shift", K + 2), ("in_scale", K + 2), ("out_shift", 3 * (K + 1) + 2),
                     ("out_scale", 3 * (K + 1) + 2)):
        word(key)
        out[key] = np.array([float(v) for v in take(cnt)], dtype=np.float32)
    word("params")
    n = int(take()[0])
    out["params"] = np.array([float(v) for v in take(n)], dtype=np.float32)
    word("end")
    return out


def network_outputs(pred: dict, states: np.ndarray) -> np.ndarray:
    """De-standardised network outputs t [n, 3N+2] for rows (T, Y, P)."""
    K = pred["K"]
    T, Y, P = states[:, 0], states[:, 1:K + 1], states[:, K + 1]
    f = np.concatenate([(T / 1000.0)[:, None], np.log(P / P_ATM)[:, None], Y], axis=1)
    x = ((f - pred["in_shift"].astype(np.float64)) / pred["in_scale"].astype(np.float64)).astype(np.float32)
    y = MlpRef(pred["dims"], pred["params"]).forward(x.astype(np.float64))
    return y * pred["out_scale"].astype(np.float64) + pred["out_shift"].astype(np.float64)


LOG2_10 = 3.321928094887362     # log2(10)


def warm_start(pred: dict, states: np.ndarray, atol: float, rtol: float, dt: float = None):
    """(h [n], z [n, 3, N], steps [n]) decoded as described in the module
    docstring; dt defaults to the global step the predictor was trained for."""
    dt = pred["dt"] if dt is None else dt
    K = pred["K"]
    N = K + 1
    n = states.shape[0]
    t = network_outputs(pred, states)
    ok = np.isfinite(t)
    t = np.where(ok, t, 0.0)
    tz = np.clip(t[:, :3 * N], -40.0, 40.0).reshape(n, 3, N)
    sc = atol + rtol * np.abs(states[:, :N])
    z = np.sign(tz) * np.expm1(np.abs(tz)) * sc[:, None, :]
    z = np.where(ok[:, :3 * N].reshape(n, 3, N), z, 0.0)
    q = np.rint(-np.clip(t[:, 3 * N], -15.0, 0.0) * LOG2_10)
    h = np.where(ok[:, 3 * N], np.ldexp(dt, (-q).astype(np.int64)), 0.0)
    steps = np.where(ok[:, 3 * N + 1], 10.0 ** np.clip(t[:, 3 * N + 1], 0.0, 7.0), 0.0)
    return h, z, steps
