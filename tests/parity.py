"""Comparison helpers shared by the GPU parity tests."""
import sys

import numpy as np

from paper_1607_03884_amd import gen

EPS = np.finfo(float).eps


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def integration_errors(got: np.ndarray, ref: np.ndarray, K: int, ythresh: float = 1e-8):
    """The acceptance metric: max relative error on T and on every Y_i whose
    oracle value exceeds `ythresh`.  Rows are (T, Y_1..Y_K, P)."""
    relT = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    Yg, Yr = got[:, 1:K + 1], ref[:, 1:K + 1]
    mask = Yr > ythresh
    relY = np.where(mask, np.abs(Yg - Yr) / np.where(mask, Yr, 1.0), 0.0)
    return float(relT.max(initial=0.0)), float(relY.max(initial=0.0))


def rhs_magnitudes(mech: gen.Mechanism, om, row: np.ndarray) -> np.ndarray:
    """Size of the terms summed into each component of f (rounding scale):
    W_k/rho sum_j |nu_kj| (|qf_j| + |qr_j|) for species (q_j = qf_j - qr_j can
    cancel near equilibrium), and the matching enthalpy-weighted sum for T."""
    K = mech.K
    y, P = row[:K + 1], row[K + 1]
    q, w, qf, qr = om.rates_fr(y, P)
    Y = y[1:]
    Wbar = 1.0 / np.sum(Y / mech.W)
    rho = P * Wbar / (gen.R_U * y[0])
    mag = np.zeros(K)
    for j, r in enumerate(mech.reactions):
        for s in (*r.reac, *r.prod):
            mag[s] += abs(qf[j]) + abs(qr[j])
    magY = mech.W * mag / rho
    cp, h, _ = om.thermo(y[0])
    cpm = np.sum(Y * cp / mech.W)
    magT = y[0] * np.sum(np.abs(h) * mag) / (rho * cpm)
    return np.concatenate([[magT], magY])
