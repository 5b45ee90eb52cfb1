"""Pins of the oracle's first-order finite-difference Jacobian (the variant the
paper compares with the analytical Jacobian, Sec. 3.4).

* For f_i(y) = sum_j A_ij y_j^2 a forward difference is exact up to the
  truncation term A_ij inc_j, so each column's increment can be read back and
  is checked against CVODE's difference-quotient rule (sqrt(u) |y_j|, floored
  by 1000 |h| u N ||f||_w w_j).
* On the chemistry the forward differences agree with the analytical
  Jacobian (itself pinned against the complex-step derivative) to first order.
* Radau IIA with the finite-difference Jacobian reaches the same solution as
  with the analytical one (simplified Newton converges to the same collocation
  solution; only the iteration differs), within the acceptance bar, and the
  closed form of a linear system.
"""
import math

import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen
from tests.parity import rhs_magnitudes

U = 2.0 ** -52


def _rule(y, f, h, atol, rtol):
    w = atol + rtol * np.abs(y)
    fn = math.sqrt(np.mean((f / w) ** 2))
    m = 1000.0 * abs(h) * U * len(y) * fn if fn != 0.0 else 1.0
    return np.maximum(math.sqrt(U) * np.abs(y), m * w)


@pytest.mark.parametrize("h", [1e-9, 1e-6, 1e-3])
def test_fd_increments_read_back_from_a_quadratic(oracle_mod, h):
    """f_i = a_i y_i^2: the forward difference of column i is a_i (2 y_i + inc_i),
    so a component with y_i = 0 gives its increment exactly (the floor
    m w_i with w_i = atol), and the others give it to the rounding of the
    difference (the sqrt(u) |y_i| regime, checked to a factor of 2)."""
    N = 9
    a = np.array([1.5, -0.8, 2.0, 1.1, -1.3, 0.9, 1.7, -0.6, 1.2])
    A = np.diag(a)
    y = np.array([3.0, -0.7, 0.0, 2e-2, 0.0, 5e-1, 40.0, 0.0, 1e-3])
    atol, rtol = 1e-10, 1e-6
    J = oracle_mod.jac_fd_quadratic(A, y, h, atol, rtol)
    f = a * y * y
    want = _rule(y, f, h, atol, rtol)
    got = np.diag(J) / a - 2.0 * y
    assert np.all(J[~np.eye(N, dtype=bool)] == 0.0)
    zero = y == 0.0
    assert np.allclose(got[zero], want[zero], rtol=1e-12, atol=0.0), (got[zero], want[zero])
    assert np.all(np.abs(got[~zero] - want[~zero]) <= 1.0 * want[~zero])
    # f(y) = 0: the floor multiplier is 1, so inc_i = w_i
    y0 = np.zeros(N)
    J0 = oracle_mod.jac_fd_quadratic(A, y0, h, atol, rtol)
    assert np.allclose(np.diag(J0) / a, atol, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("mname", ["m13", "m53"])
def test_fd_jacobian_matches_analytical_to_first_order(request, mname):
    """Columns whose increment is sqrt(u) |y_j| agree to ~1e-5 of the row
    scale; columns on the increment floor (trace species, where inc_j / |y_j|
    can reach a few per cent) to within that relative perturbation."""
    m = request.getfixturevalue(mname)
    st = gen.uniform_states(m.K, 6, 41)
    h = 1e-13        # the size of these far-from-equilibrium states' first steps
    worst = 0.0
    for row in st:
        y, P = row[:m.N], row[-1]
        J = m.jac(y, P)
        Jfd = m.jac_fd(y, P, h)
        inc = _rule(y, m.rhs(y, P), h, 1e-10, 1e-6)
        rel = inc / np.maximum(np.abs(y), 1e-300)
        scale = np.abs(J).max(axis=1, keepdims=True) + 1e-300
        dev = np.abs(Jfd - J) / scale
        # rounding of the quotient: u times the size of the terms summed into f_i, over inc_j
        mech = gen.make_mechanism(configs.MECHS["M13" if m.K == 13 else "M53"])
        mag = rhs_magnitudes(mech, m, row)
        rnd = 64 * U * mag[:, None] / inc[None, :] / scale
        sqrt_regime = np.isclose(inc, math.sqrt(U) * np.abs(y), rtol=1e-12, atol=0.0)
        assert np.all((dev - rnd)[:, sqrt_regime] <= 1e-4), (dev - rnd)[:, sqrt_regime].max()
        assert np.all(dev <= 3.0 * rel[None, :] + rnd + 1e-4)
        worst = max(worst, float(dev.max()))
    assert worst > 1e-14          # it is a difference quotient, not the analytical matrix


@pytest.mark.parametrize("dt", [1e-6, 1e-4])
def test_radau_with_fd_jacobian_reaches_the_same_solution(m13, dt):
    from oracle import default_opts
    rows = configs.states_for(configs.WORKLOADS["cfg1"], 96)
    a, ra = m13.integrate(rows, dt)
    b, rb = m13.integrate(rows, dt, opts=default_opts(fd_jac=1))
    assert np.all(ra["status"] == 0) and np.all(rb["status"] == 0)
    relT = np.abs(b[:, 0] - a[:, 0]) / a[:, 0]
    Ya, Yb = a[:, 1:14], b[:, 1:14]
    mask = Ya > 1e-8
    relY = np.abs(Yb - Ya)[mask] / Ya[mask]
    assert relT.max() <= 1e-5 and relY.max() <= 1e-4
    # each finite-difference Jacobian costs N source-term evaluations (states
    # whose step, Jacobian, Newton and rejection counts agree)
    same = np.ones(len(rows), dtype=bool)
    for k in ("nstep", "njev", "nnewton", "nreject"):
        same &= ra[k] == rb[k]
    assert same.mean() >= 0.5
    extra = (rb["nfev"] - ra["nfev"])[same]
    assert np.mean(extra == 14 * rb["njev"][same]) >= 0.95


def test_fd_jacobian_on_linear_system_closed_form(oracle_mod):
    """y' = M y: the Radau IIA solution with the finite-difference Jacobian
    matches exp(M dt) y0 to the tolerance."""
    from scipy.linalg import expm
    from oracle import default_opts
    rng = np.random.default_rng(8)
    N = 6
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    lam = -np.logspace(0, 6, N)
    M = Q @ np.diag(lam) @ Q.T
    y0 = rng.standard_normal(N)
    dt = 1e-2
    out, res, _ = oracle_mod.integrate_linear(M, y0, dt, 1e-12, 1e-9, opts=default_opts(fd_jac=1))
    want = expm(M * dt) @ y0
    assert res.status == 0
    assert np.abs(out - want).max() <= 1e-7 * np.abs(y0).max()
