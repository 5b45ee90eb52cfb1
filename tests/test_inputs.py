"""The seeded synthetic inputs checked against the recipe they are built to.

Mechanisms: sizes, reaction kinds, element balance, molar masses from the
element compositions, and parameter ranges, with every reaction written in
its exothermic direction.  State sets: shapes, ranges, the fresh/burnt mix of
the PaSR-like sets, and determinism.  These inputs stand in for the paper's
hydrogen and methane models and PaSR databases (Sec. 2.2), which are not
available here.
"""
import numpy as np
import pytest

from paper_1607_03884_amd import configs, gen

KCAL = 1000.0 * gen.CAL


@pytest.fixture(scope="module", params=["M13", "M53", "M150"])
def mech(request):
    return request.param, gen.make_mechanism(configs.MECHS[request.param])


def test_sizes_and_reaction_kinds(mech):
    name, m = mech
    spec = configs.MECHS[name]
    assert len(m.species) == spec.n_species
    assert len(m.reactions) == spec.n_reactions
    kinds = [r.kind for r in m.reactions]
    n3 = spec.n_three_body if spec.n_three_body is not None else round(spec.frac_three_body * spec.n_reactions)
    nt = spec.n_troe if spec.n_troe is not None else round(spec.frac_troe * spec.n_reactions)
    assert kinds.count(gen.THREE_BODY) == n3
    assert kinds.count(gen.TROE) == nt
    assert kinds.count(gen.ELEMENTARY) == spec.n_reactions - n3 - nt
    assert set(kinds) <= {gen.ELEMENTARY, gen.THREE_BODY, gen.TROE}


def test_balance_species_use_and_molar_masses(mech):
    name, m = mech
    K = len(m.species)
    inert = set(m.inert)
    used = set()
    for r in m.reactions:
        assert 1 <= len(r.reac) <= 2 and 1 <= len(r.prod) <= 2
        assert np.array_equal(m.comp[list(r.reac)].sum(axis=0), m.comp[list(r.prod)].sum(axis=0))
        used |= set(r.reac) | set(r.prod)
    assert not (used & inert)
    assert used == set(range(K)) - inert              # every active species takes part
    W = np.array([sum(m.comp[k, e] * gen.ATOMIC_WEIGHT[el] for e, el in enumerate(m.elements))
                  for k in range(K)]) * 1e-3
    np.testing.assert_allclose(m.W, W, rtol=1e-12)


def test_parameter_ranges(mech):
    name, m = mech
    K = len(m.species)
    for r in m.reactions:
        order = len(r.reac) + (1 if r.kind == gen.THREE_BODY else 0)
        A_cgs = r.A / (1e-6) ** (order - 1)
        assert 1e6 * (1 - 1e-12) <= A_cgs <= 1e14 * (1 + 1e-12)
        assert -1.5 <= r.b <= 2.0
        assert 0.0 <= r.Ea <= 40.0 * KCAL
        if r.kind == gen.TROE:
            assert 1e-3 * (1 - 1e-12) <= r.A0 / r.A <= 10.0 * (1 + 1e-12)     # 10^U[3,7] cm^3/mol in SI
            assert r.b0 == r.b and r.Ea0 == r.Ea
            a, t3, t1, t2 = r.troe
            assert 0.3 <= a <= 0.9 and 10.0 <= t3 <= 1000.0
            assert 500.0 <= t1 <= 5000.0 and 1000.0 <= t2 <= 10000.0
        else:
            assert r.A0 == 0.0 and r.troe == (0.0, 0.0, 0.0, 0.0)
        if r.kind == gen.ELEMENTARY:
            assert not r.eff
        for k, e in r.eff.items():
            assert 0 <= k < K and 0.4 <= e <= 6.0


def _h_over_R(a, T):
    return T * (a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5) + a[5]


def test_reactions_written_exothermic(mech):
    """Enthalpy of reaction at 298.15 K from the low-range NASA-7 fits is not
    positive (the generator orients each reaction by heats of formation)."""
    name, m = mech
    T = 298.15
    h = np.array([_h_over_R(m.a_low[k], T) for k in range(len(m.species))]) * gen.R_U
    for r in m.reactions:
        dH = h[list(r.prod)].sum() - h[list(r.reac)].sum()
        assert dH <= 1e-6 * (1.0 + np.abs(h[list(r.prod) + list(r.reac)]).max())


def _check_rows(s, K):
    assert s.shape[1] == K + 2
    Y = s[:, 1:K + 1]
    assert np.all(np.isfinite(s))
    assert Y.min() >= 0.0
    np.testing.assert_allclose(Y.sum(axis=1), 1.0, rtol=0, atol=1e-12)
    P_atm = s[:, K + 1] / gen.P_ATM
    assert P_atm.min() >= 1.0 * (1 - 1e-12) and P_atm.max() <= 25.0 * (1 + 1e-12)


def test_uniform_state_set():
    wl = configs.WORKLOADS["cfg0"]
    K = configs.MECHS[wl.mech].n_species
    s = configs.states_for(wl)
    assert s.shape[0] == wl.n_states
    _check_rows(s, K)
    assert s[:, 0].min() >= 900.0 and s[:, 0].max() <= 2200.0
    assert np.array_equal(s, configs.states_for(wl))


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg4"])
def test_pasr_like_state_sets(name):
    wl = configs.WORKLOADS[name]
    K = configs.MECHS[wl.mech].n_species
    tpl = configs.load_templates(wl.mech)
    assert tpl.shape == (configs.N_TEMPLATES, K + 2)
    _check_rows(tpl, K)
    assert tpl[:, 0].min() >= 1800.0 and tpl[:, 0].max() <= 2400.0
    s = configs.states_for(wl)
    assert s.shape[0] == wl.n_states
    _check_rows(s, K)
    T = s[:, 0]
    fresh = (T >= 900.0) & (T <= 1200.0)
    burnt = (T >= 1800.0) & (T <= 2400.0)
    assert np.all(fresh | burnt)
    assert fresh.sum() == round(0.3 * wl.n_states)
    # shuffled: every group of 64 consecutive states holds both kinds
    m = (wl.n_states // 64) * 64
    f64 = fresh[:m].reshape(-1, 64)
    assert f64.any(axis=1).all() and (~f64).any(axis=1).all()
    # burnt states keep their template's T and P; only Y is perturbed
    tp = {(t, p) for t, p in zip(tpl[:, 0], tpl[:, K + 1])}
    assert all((t, p) in tp for t, p in zip(s[burnt, 0][:2000], s[burnt, K + 1][:2000]))
    assert np.array_equal(configs.states_for(wl, 1000), s[:1000])
