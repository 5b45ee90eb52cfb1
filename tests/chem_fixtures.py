"""Small hand-built mechanisms for closed-form checks (written through the same
text format the generators use)."""
import numpy as np

from paper_1607_03884_amd import gen


def const_cp_coeffs(cp_over_R: float, h_over_R_const: float, s_const: float):
    a = np.zeros(7)
    a[0] = cp_over_R
    a[5] = h_over_R_const
    a[6] = s_const
    return a


def mini_mech(species, reactions, W=None, thermo=None, name="mini"):
    """species: list of (name, {elem: n}); reactions: list of gen.Reaction;
    thermo: list of (a_low, a_high) per species (defaults: cp/R = 3.5)."""
    elements = sorted({e for _, c in species for e in c})
    K = len(species)
    comp = np.array([[c.get(e, 0) for e in elements] for _, c in species], dtype=np.int64)
    if W is None:
        W = np.array([sum(gen.ATOMIC_WEIGHT[e] * n for e, n in c.items()) for _, c in species]) * 1e-3
    a_low = np.zeros((K, 7))
    a_high = np.zeros((K, 7))
    for k in range(K):
        if thermo is None:
            a_low[k] = a_high[k] = const_cp_coeffs(3.5, 0.0, 20.0)
        else:
            a_low[k], a_high[k] = thermo[k]
    return gen.Mechanism(name, elements, [n for n, _ in species], comp, np.asarray(W, dtype=float),
                         np.full(K, 300.0), np.full(K, 1000.0), np.full(K, 6000.0), a_low, a_high,
                         list(reactions), [])


def write(m, tmp_path, fname="mini.mech"):
    p = tmp_path / fname
    p.write_text(gen.mech_text(m))
    return str(p)
