"""Pins of the oracle's Radau IIA coefficients against the defining conditions
(Hairer & Wanner's three-stage Radau IIA, cited in Sec. 2.1): simplifying
assumptions B(5), C(3), D(2) and the failure of the next order of each, the
stability function as the (2,3) Pade approximant of exp, the eigen-structure
used by the transformed Newton iteration, and the embedded error estimate
rebuilt from its order conditions."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def K(oracle_mod):
    return oracle_mod.radau_constants()


def test_simplifying_assumptions(K):
    A, b, c = K["A"], K["b"], K["c"]
    # B(5): sum_i b_i c_i^(k-1) = 1/k, k = 1..5 ; B(6) fails
    for k in range(1, 6):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-15
    assert abs(b @ c ** 5 - 1.0 / 6) > 1e-4
    # C(3): sum_j a_ij c_j^(k-1) = c_i^k / k ; C(4) fails
    for k in range(1, 4):
        assert np.abs(A @ c ** (k - 1) - c ** k / k).max() < 1e-15
    assert np.abs(A @ c ** 3 - c ** 4 / 4).max() > 1e-4
    # D(2): sum_i b_i c_i^(k-1) a_ij = b_j (1 - c_j^k)/k ; D(3) fails
    for k in range(1, 3):
        assert np.abs((b * c ** (k - 1)) @ A - b * (1 - c ** k) / k).max() < 1e-15
    assert np.abs((b * c ** 2) @ A - b * (1 - c ** 3) / 3).max() > 1e-4
    # stiffly accurate: b is the last row of A, c_3 = 1
    assert np.array_equal(b, A[2]) and c[2] == 1.0


def test_stability_function_is_pade23(K):
    A, b = K["A"], K["b"]
    for z in [-1.0, -10.0, -1e3, -1e8, 0.5, -2.0 + 3.0j]:
        R = 1.0 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))
        pade = (1 + 2 * z / 5 + z * z / 20) / (1 - 3 * z / 5 + 3 * z * z / 20 - z ** 3 / 60)
        assert abs(R - pade) <= 1e-13 * max(1.0, abs(pade))


def test_eigenstructure_and_transformation(K):
    A = K["A"]
    Ainv = np.linalg.inv(A)
    ev = np.linalg.eigvals(Ainv)
    real = ev[np.abs(ev.imag) < 1e-12].real
    cplx = ev[ev.imag > 1e-12]
    assert abs(real[0] - K["gamma"]) < 1e-13
    assert abs(cplx[0].real - K["alpha"]) < 1e-13 and abs(cplx[0].imag - K["beta"]) < 1e-13
    # values quoted to 10 digits in the design notes
    assert abs(K["gamma"] - 3.6378342527) < 1e-10
    assert abs(K["alpha"] - 2.6810828736) < 1e-10 and abs(K["beta"] - 3.0504301992) < 1e-10
    T, Ti = K["T"], K["Tinv"]
    assert np.abs(T @ Ti - np.eye(3)).max() < 1e-13
    Lam = Ti @ Ainv @ T
    want = np.array([[K["gamma"], 0, 0], [0, K["alpha"], -K["beta"]], [0, K["beta"], K["alpha"]]])
    assert np.abs(Lam - want).max() < 1e-12


def test_error_estimate_weights_from_order_conditions(K):
    """The embedded solution y^ = y0 + h (g0 f(x0, y0) + sum_i bh_i f(x0 + c_i h, Y_i)),
    g0 = 1/gamma, of order 3 gives err = g0 h f0 + sum_i e_i z_i with
    e = (bh - b)^T A^-1; the oracle stores d = e / g0."""
    A, b, c = K["A"], K["b"], K["c"]
    g0 = 1.0 / K["gamma"]
    V = np.vstack([np.ones(3), c, c * c])
    rhs = np.array([1.0 - g0, 0.5, 1.0 / 3.0])
    bh = np.linalg.solve(V, rhs)
    e = (bh - b) @ np.linalg.inv(A)
    assert np.abs(e / g0 - K["d"]).max() < 1e-12
    assert np.abs(e - np.array([-2.76230545, 0.3799356, -0.09162961])).max() < 1e-7
