"""Pins of the oracle's rate constants against facts that do not depend on how
the oracle writes them (paper Sec. 2.1: the source terms and analytical
Jacobian come from a reversible mass-action model with third-body and falloff
reactions).

* Arrhenius law: ln k_f is linear in (1, ln T, 1/T) with coefficients
  (ln A, b, -E_a/R); recovered by least squares over six temperatures, and
  the relaxation of an isomerisation with b != 0, E_a != 0 against its
  closed form.
* Equilibrium constant: at a composition that satisfies the Gibbs condition
  sum_k nu_k (g_k/RT + ln(X_k P/P_atm)) = 0 (computed from the test's own
  constant-c_p thermodynamics), forward and reverse rates are equal, for a
  dissociation (sum nu = +1) and a recombination (sum nu = -1), elementary,
  third-body and falloff.
* Troe blending: at the pressures where f1 = 0, +1, -1, +2 the blend is
  F_cent, F_cent^(1/2), F_cent^(1/2), F_cent^(1/5), for four choices of the
  Troe parameters that make each term of F_cent known exactly.
"""
import math

import numpy as np
import pytest

from paper_1607_03884_amd import gen
from tests import chem_fixtures as cf

RU = gen.R_U
PATM = 101325.0


def _conc(mech, y, P):
    Y = y[1:]
    Wbar = 1.0 / np.sum(Y / mech.W)
    rho = P * Wbar / (RU * y[0])
    return rho * Y / mech.W


def _isomer_mech(A, b, Ea):
    aA = cf.const_cp_coeffs(4.0, -5000.0, 10.0)
    aB = cf.const_cp_coeffs(4.0, -5000.0, 10.7)
    sp = [("CO", {"C": 1, "O": 1}), ("OC", {"C": 1, "O": 1}), ("N2", {"N": 2})]
    rx = [gen.Reaction(gen.ELEMENTARY, (0,), (1,), A, b, Ea)]
    return cf.mini_mech(sp, rx, thermo=[(aA, aA), (aB, aB), (aA, aA)])


def _kf(m, mech, T, P=2e5):
    # pure reactant side (no product): q = k_f C_A
    y = np.array([T, 0.4, 0.0, 0.6])
    q, _ = m.rates(y, P)
    return q[0] / _conc(mech, y, P)[0]


@pytest.mark.parametrize("A,b,Ea", [(3.0e6, 0.0, 80e3), (3.0e6, 1.5, 0.0), (7.5e9, 1.5, 80e3), (2.0e4, -1.2, 1.5e5)])
def test_arrhenius_coefficients_recovered(oracle_mod, tmp_path, A, b, Ea):
    mech = _isomer_mech(A, b, Ea)
    m = oracle_mod.Mech(cf.write(mech, tmp_path))
    T = np.array([700.0, 950.0, 1300.0, 1650.0, 2100.0, 2600.0])
    lk = np.log([_kf(m, mech, t) for t in T])
    X = np.stack([np.ones_like(T), np.log(T), 1.0 / T], axis=1)
    coef, *_ = np.linalg.lstsq(X, lk, rcond=None)
    assert abs(coef[0] - math.log(A)) <= 1e-9 * max(1.0, abs(math.log(A)))
    assert abs(coef[1] - b) <= 1e-9
    assert abs(coef[2] + Ea / RU) <= 1e-9 * max(1.0, Ea / RU)
    assert np.abs(X @ coef - lk).max() <= 1e-12 * np.abs(lk).max()


def test_isomerisation_closed_form_with_temperature_dependence(oracle_mod, tmp_path):
    """A <=> B relaxes at k_f + k_r with k_f = A T^b exp(-E_a/RT); equal h and
    c_p keep T constant, K_c = exp(s_B/R - s_A/R)."""
    A, b, Ea = 1.0e5, 1.5, 80e3
    mech = _isomer_mech(A, b, Ea)
    m = oracle_mod.Mech(cf.write(mech, tmp_path))
    st = np.array([[1500.0, 0.6, 0.1, 0.3, 2e5], [1100.0, 0.05, 0.9, 0.05, 1e6]])
    dt = 2e-7
    out, res = m.integrate(st, dt, atol=1e-12, rtol=1e-9)
    assert np.all(res["status"] == 0)
    for s, o in zip(st, out):
        kf = A * s[0] ** b * math.exp(-Ea / (RU * s[0]))
        kr = kf / math.exp(10.7 - 10.0)
        tot = s[1] + s[2]
        yeq = kr / (kf + kr) * tot
        want = yeq + (s[1] - yeq) * math.exp(-(kf + kr) * dt)
        assert 0.1 < (kf + kr) * dt < 5.0      # the relaxation is under way, not finished
        assert abs(o[0] - s[0]) <= 1e-9 * s[0]
        assert abs(o[1] - want) <= 1e-7 * abs(want)


# ---- equilibrium constant -----------------------------------------------------------

def _dissociation_mech(kind, forward_dissociation, b=0.7, Ea=4e4):
    # H2 <=> 2 H (sum nu = +1) or 2 H <=> H2 (sum nu = -1); constant c_p thermo
    aH = cf.const_cp_coeffs(2.5, 26000.0, -0.5)
    aH2 = cf.const_cp_coeffs(3.5, -1000.0, -1.2)
    aAr = cf.const_cp_coeffs(2.5, -745.0, 4.4)
    sp = [("H", {"H": 1}), ("H2", {"H": 2}), ("Ar", {"Ar": 1})]
    reac, prod = ((1,), (0, 0)) if forward_dissociation else ((0, 0), (1,))
    kw = {}
    if kind == gen.TROE:
        kw = dict(A0=3.0e3, b0=-0.5, Ea0=1e3, troe=(0.6, 200.0, 1500.0, 4000.0), eff={2: 0.6})
    elif kind == gen.THREE_BODY:
        kw = dict(eff={1: 2.5, 2: 0.8})
    r = gen.Reaction(kind, reac, prod, 4.0e5, b, Ea, **kw)
    mech = cf.mini_mech(sp, [r], thermo=[(aH, aH), (aH2, aH2), (aAr, aAr)])
    return mech, (aH, aH2, aAr)


def _g_over_RT(a, T):
    # constant c_p: h/RT = a1 + a6/T, s/R = a1 ln T + a7
    return a[0] + a[5] / T - (a[0] * math.log(T) + a[6])


def _equilibrium_state(coeffs, T, P, x_ar=0.5):
    aH, aH2, _ = coeffs
    dG = 2.0 * _g_over_RT(aH, T) - _g_over_RT(aH2, T)      # H2 -> 2 H
    Kx = math.exp(-dG) * PATM / P                            # X_H^2 / X_H2
    tot = 1.0 - x_ar
    xh = 0.5 * (-Kx + math.sqrt(Kx * Kx + 4.0 * Kx * tot))
    return np.array([xh, tot - xh, x_ar])


@pytest.mark.parametrize("kind", [gen.ELEMENTARY, gen.THREE_BODY, gen.TROE])
@pytest.mark.parametrize("forward_dissociation", [True, False])
def test_equilibrium_constant_satisfies_gibbs_condition(oracle_mod, tmp_path, kind, forward_dissociation):
    mech, coeffs = _dissociation_mech(kind, forward_dissociation)
    m = oracle_mod.Mech(cf.write(mech, tmp_path))
    for T, P in ((2200.0, 1e5), (3000.0, 2.5e6), (2600.0, 4e3)):
        X = _equilibrium_state(coeffs, T, P)
        assert 1e-6 < X[0] < 0.5 - 1e-6                       # both sides present
        Y = X * mech.W / np.sum(X * mech.W)
        y = np.concatenate([[T], Y])
        q, _, qf, qr = m.rates_fr(y, P)
        assert abs(q[0]) <= 1e-11 * qf[0], (T, P, q[0] / qf[0])
        # off equilibrium the net rate has the sign the Gibbs condition gives
        Xo = X.copy()
        Xo[0] *= 1.2
        Xo[1] -= X[0] * 0.2
        Yo = Xo * mech.W / np.sum(Xo * mech.W)
        q2, _, qf2, _ = m.rates_fr(np.concatenate([[T], Yo]), P)
        # excess H drives recombination: H2 -> 2 H runs backward, 2 H -> H2 forward
        assert (q2[0] < 0) == forward_dissociation
        assert abs(q2[0]) > 1e-3 * qf2[0]


# ---- Troe blending --------------------------------------------------------------------

def _troe_cases(T):
    # (a, T***, T*, T**) and the F_cent each gives exactly
    return [((1.0, 1000.0, T / math.log(2.0), 1e300), 0.5),
            ((0.0, T / math.log(4.0), 1000.0, 1e300), 0.25),
            ((0.0, 1e-300, 1000.0, T * math.log(5.0)), 0.2),
            ((0.4, T / math.log(2.0), T / math.log(4.0), T * math.log(10.0)), 0.6 * 0.5 + 0.4 * 0.25 + 0.1)]


@pytest.mark.parametrize("case", range(4))
def test_troe_blend_at_known_points(oracle_mod, tmp_path, case):
    T = 1400.0
    troe, Fc = _troe_cases(T)[case]
    kinf, k0 = 2.0e5, 3.0e3
    sp = [("H", {"H": 1}), ("H2", {"H": 2}), ("Ar", {"Ar": 1})]
    r_ref = gen.Reaction(gen.ELEMENTARY, (0, 0), (1,), kinf, 0.0, 0.0)
    r = gen.Reaction(gen.TROE, (0, 0), (1,), kinf, 0.0, 0.0, A0=k0, troe=troe)
    mech = cf.mini_mech(sp, [r_ref, r])
    m = oracle_mod.Mech(cf.write(mech, tmp_path))
    L = math.log10(Fc)
    c = -0.4 - 0.67 * L
    n = 0.75 - 1.27 * L
    # log10 Pr + c = x with f1 = x / (n - 0.14 x) taking the values 0, 1, -1, 2
    for f1, F in ((0.0, Fc), (1.0, Fc ** 0.5), (-1.0, Fc ** 0.5), (2.0, Fc ** 0.2)):
        x = f1 * n / (1.0 + 0.14 * f1)
        Pr = 10.0 ** (x - c)
        P = Pr * kinf / k0 * RU * T          # [M] = P/(R T) with unit efficiencies
        y = np.array([T, 0.1, 0.2, 0.7])
        q, _ = m.rates(y, P)
        ratio = q[1] / q[0]
        want = Pr / (1.0 + Pr) * F
        assert abs(ratio - want) <= 1e-11 * want, (case, f1, ratio, want)
