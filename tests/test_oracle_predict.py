"""Pins of the CPU warm-start decoder (oracle/predict.py): a network whose
weights are all zero outputs its de-standardisation shift, so every decoded
value has a closed form written out here; the committed predictor files
parse and fit their mechanism."""
import os

import numpy as np
import pytest

from oracle import predict
from paper_1607_03884_amd import configs, predictor as trainer


def _zero_net(tmp_path, K, dt, out_shift):
    N = K + 1
    dims = [K + 2, 8, 3 * N + 2]
    nparam = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(2))
    path = os.path.join(str(tmp_path), "zero.rkp")
    trainer.write(path, "T", K, dt, dims, np.zeros(K + 2), np.ones(K + 2), out_shift, np.ones(3 * N + 2),
                  np.zeros(nparam))
    return predict.load(path)


def test_decode_closed_forms(tmp_path):
    K, dt = 2, 1e-6
    N = K + 1
    shift = np.zeros(3 * N + 2)
    shift[0], shift[1], shift[N + 2] = 1.0, -2.0, 45.0     # z_00, z_01, z_12 (clipped at 40)
    shift[3 * N] = -3.0                                        # log10(h/dt) = -3 -> q = round(9.966) = 10
    shift[3 * N + 1] = 2.0                                     # 100 step attempts
    pr = _zero_net(tmp_path, K, dt, shift.astype(np.float32))
    st = np.array([[1500.0, 0.25, 0.75, 2e5]])
    h, z, steps = predict.warm_start(pr, st, 1e-10, 1e-6)
    sc = 1e-10 + 1e-6 * np.abs(st[0, :N])
    assert h[0] == dt / 1024.0
    assert np.isclose(steps[0], 100.0, rtol=1e-6)
    assert np.isclose(z[0, 0, 0], (np.e - 1.0) * sc[0], rtol=1e-12)
    assert np.isclose(z[0, 0, 1], -(np.e ** 2 - 1.0) * sc[1], rtol=1e-12)
    assert np.isclose(z[0, 1, 2], (np.exp(40.0) - 1.0) * sc[2], rtol=1e-12)
    assert z[0, 2, 0] == 0.0


@pytest.mark.parametrize("t,q", [(0.0, 0), (0.5, 0), (-0.15, 0), (-0.16, 1), (-1.0, 3), (-20.0, 50)])
def test_first_step_rounding(tmp_path, t, q):
    """h = dt 2^-q with q the nearest integer to -log2(10) t (t clipped to [-15, 0])."""
    K, dt = 1, 1e-4
    shift = np.zeros(3 * (K + 1) + 2, dtype=np.float32)
    shift[3 * (K + 1)] = t
    pr = _zero_net(tmp_path, K, dt, shift)
    h, _, _ = predict.warm_start(pr, np.array([[1000.0, 1.0, 1e5]]), 1e-10, 1e-6)
    assert h[0] == np.ldexp(dt, -q)


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
def test_committed_predictors_parse(dt):
    pr = predict.load(trainer.path_for("M13", dt))
    assert pr["K"] == 13 and pr["dims"][0] == 15 and pr["dims"][-1] == 3 * 14 + 2
    assert pr["dt"] == dt
    st = configs.states_for(configs.WORKLOADS["cfg0"], 32)
    h, z, steps = predict.warm_start(pr, st, 1e-10, 1e-6)
    assert np.all(h > 0) and np.all(h <= dt) and np.all(np.isfinite(z)) and np.all(steps >= 1)
    # every h is dt times a power of two
    m, e = np.frexp(h / dt)
    assert np.all(m == 0.5)
