"""Pins of the oracle's Rosenbrock integrator (Rodas3), the semi-implicit
method the paper's conclusions recommend (Sec. 4).

* The stored coefficient table (transformed form: gamma, a, c, m, e) is
  converted back to the classical form (alpha, Gamma, b) and checked against
  the Rosenbrock order conditions: all of order <= 3 hold, order 4 fails; the
  embedded weights m - e satisfy those of order <= 2.
* One step on y' = lambda y equals the stability function
  R(z) = 1 + z b^T (I - z (alpha + Gamma))^-1 1 of that table, which is
  L-stable (R(-inf) = 0) and agrees with e^z to O(z^4).
* Fixed steps on the chemistry converge at order 3.
* Linear invariants (sum of Y, element totals) are kept to rounding, and an
  isomerisation matches its closed form.
"""
import math

import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen
from tests import chem_fixtures as cf


def _classical(t):
    g = t["gamma"]
    A, C = np.tril(t["a"], -1), np.tril(t["c"], -1)
    Gam = np.linalg.inv(np.diag(np.full(4, 1.0 / g)) - C)
    alpha = A @ Gam
    return g, alpha, Gam, t["m"] @ Gam, (t["m"] - t["e"]) @ Gam


def _conditions(b, alpha, Gam, g):
    beta = np.tril(alpha + Gam, -1)
    a_i, b_i = alpha.sum(1), beta.sum(1)
    return np.array([b.sum() - 1.0,
                     b @ b_i - (0.5 - g),
                     b @ a_i ** 2 - 1.0 / 3.0,
                     b @ (beta @ b_i) - (1.0 / 6.0 - g + g * g),
                     b @ a_i ** 3 - 0.25,
                     b @ (a_i * (alpha @ b_i)) - (1.0 / 8.0 - g / 3.0),
                     b @ (beta @ a_i ** 2) - (1.0 / 12.0 - g / 3.0),
                     b @ (beta @ (beta @ b_i)) - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3)])


def test_rodas3_table_order_conditions(oracle_mod):
    t = oracle_mod.rodas3_table()
    g, alpha, Gam, b, bhat = _classical(t)
    assert np.allclose(np.diag(Gam), g, rtol=0, atol=1e-15)
    c = _conditions(b, alpha, Gam, g)
    assert np.all(np.abs(c[:4]) <= 1e-14), c
    assert np.abs(c[4:]).max() > 1e-3                  # order exactly 3
    ch = _conditions(bhat, alpha, Gam, g)
    assert np.all(np.abs(ch[:2]) <= 1e-14) and np.abs(ch[2:4]).max() > 1e-3    # embedded order 2


def test_rodas3_linear_step_is_the_stability_function(oracle_mod):
    t = oracle_mod.rodas3_table()
    g, alpha, Gam, b, _ = _classical(t)
    B = alpha + Gam
    R = lambda z: 1.0 + z * (b @ np.linalg.solve(np.eye(4) - z * B, np.ones(4)))
    for lam, h in ((-1.0, 0.5), (-1e3, 1e-2), (-1e8, 1.0), (0.3, 0.2)):
        y1 = oracle_mod.rodas3_linear_step(np.array([[lam]]), np.array([2.0]), h)
        assert abs(y1[0] / 2.0 - R(lam * h)) <= 1e-13 * max(1.0, abs(R(lam * h)))
    assert abs(R(-1e12)) < 1e-9                                      # L-stable
    for z in (1e-2, -1e-2):
        assert abs(R(z) - math.exp(z)) <= 2 * abs(z) ** 4           # order 3
    # a 3x3 system: the step acts through (I - z B)^-1 on each eigenvalue
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    lam = np.array([-2.0, -50.0, -4e4])
    M = Q @ np.diag(lam) @ Q.T
    y0 = rng.standard_normal(3)
    h = 0.05
    y1 = oracle_mod.rodas3_linear_step(M, y0, h)
    want = Q @ (np.array([R(l * h) for l in lam]) * (Q.T @ y0))
    assert np.abs(y1 - want).max() <= 1e-12 * np.abs(y0).max()


def test_rodas3_fixed_step_order_three(m13):
    row = configs.states_for(configs.WORKLOADS["cfg1"], 8)[3]
    dt = 2e-8
    ref, _ = m13.integrate(row[None, :], dt, atol=1e-20, rtol=1e-13)
    errs = []
    for n in (8, 16, 32):
        y = m13.rodas3_fixed_steps(row, dt, n)
        errs.append(np.abs(y - ref[0, :14]).max())
    p1, p2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 2.6 <= p2 <= 3.6 and 2.4 <= p1 <= 3.8, (errs, p1, p2)


def test_rodas3_invariants_and_isomerisation(oracle_mod, m13, tmp_path):
    mech = gen.make_mechanism(configs.MECHS["M13"])
    st = gen.uniform_states(13, 32, 33)
    out, res = m13.integrate_rodas3(st, 1e-6)
    assert np.all(res["status"] == 0) and np.all(res["nnewton"] == 0)
    assert np.abs(out[:, 1:14].sum(1) - st[:, 1:14].sum(1)).max() <= 1e-13
    U = mech.comp.T / mech.W[None, :]
    assert np.all(np.abs(out[:, 1:14] @ U.T - st[:, 1:14] @ U.T) <= 1e-12 * np.abs(st[:, 1:14] @ U.T) + 1e-12)
    # A <=> B, equal h and c_p (T constant), closed-form relaxation
    aA = cf.const_cp_coeffs(4.0, -5000.0, 10.0)
    aB = cf.const_cp_coeffs(4.0, -5000.0, 10.7)
    sp = [("CO", {"C": 1, "O": 1}), ("OC", {"C": 1, "O": 1}), ("N2", {"N": 2})]
    kf = 3.0e6
    m = oracle_mod.Mech(cf.write(cf.mini_mech(sp, [gen.Reaction(gen.ELEMENTARY, (0,), (1,), kf, 0.0, 0.0)],
                                              thermo=[(aA, aA), (aB, aB), (aA, aA)]), tmp_path))
    kr = kf / math.exp(0.7)
    s0 = np.array([[1500.0, 0.6, 0.1, 0.3, 2e5]])
    dt = 2e-7
    o, r = m.integrate_rodas3(s0, dt, atol=1e-14, rtol=1e-10)
    yeq = kr / (kf + kr) * 0.7
    want = yeq + (0.6 - yeq) * math.exp(-(kf + kr) * dt)
    assert r["status"][0] == 0
    assert abs(o[0, 1] - want) <= 1e-7 * want and abs(o[0, 0] - 1500.0) <= 1e-9 * 1500.0
