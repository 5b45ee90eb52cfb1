"""Seeded synthetic inputs: mechanisms and thermochemical states.

The paper measures on real mechanisms (a 13-species hydrogen model and the
53-species methane model, Sec. 2.2) and on partially-stirred-reactor (PaSR)
state databases (Sec. 2.2, Table 2).  Neither is available here, so this module
builds seeded stand-ins with the same shapes:

* a mechanism = species (element composition, molar mass, two-range NASA-7
  polynomials), reversible reactions with 1-2 species per side (elementary,
  third-body, Troe falloff), Arrhenius parameters drawn from the stated
  distributions;
* states = (T, Y_1..Y_K, P) rows.

This module holds data construction only (drawing parameters and fitting
polynomial coefficients to a smooth heat-capacity model); it evaluates no
source term, rate or Jacobian, and both the HIP path and the CPU oracle read
what it writes.  The text mechanism format is documented in `write_mech`.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

R_U = 8.314462618          # J/(mol K)
P_ATM = 101325.0           # Pa
CAL = 4.184                # J/cal

ATOMIC_WEIGHT = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "Ar": 39.948}  # g/mol

# Element compositions of the 13-species H2/CO-like set (chemistry facts only;
# every numeric parameter below is synthetic).
M13_SPECIES = [
    ("H", {"H": 1}), ("H2", {"H": 2}), ("O", {"O": 1}), ("O2", {"O": 2}),
    ("OH", {"O": 1, "H": 1}), ("H2O", {"H": 2, "O": 1}), ("HO2", {"H": 1, "O": 2}),
    ("H2O2", {"H": 2, "O": 2}), ("CO", {"C": 1, "O": 1}), ("CO2", {"C": 1, "O": 2}),
    ("HCO", {"H": 1, "C": 1, "O": 1}), ("CH2O", {"C": 1, "H": 2, "O": 1}),
    ("N2", {"N": 2}),
]
ELEMENT_REFERENCE = {"H2", "O2", "N2", "Ar"}

ELEMENTARY, THREE_BODY, TROE = 0, 1, 2

# bound on synthetic heats of formation (J/mol): keeps reaction enthalpies and
# equilibrium constants moderate, so adiabatic temperatures stay physical
HF_RANGE = 120e3


@dataclasses.dataclass
class Reaction:
    kind: int                      # ELEMENTARY / THREE_BODY / TROE
    reac: Tuple[int, ...]          # species index per reactant slot (1 or 2)
    prod: Tuple[int, ...]          # species index per product slot (1 or 2)
    A: float                       # SI: (m^3/mol)^(order-1)/s (high-pressure limit for TROE)
    b: float
    Ea: float                      # J/mol
    A0: float = 0.0                # TROE low-pressure limit (SI, order+1)
    b0: float = 0.0
    Ea0: float = 0.0
    troe: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)  # a, T***, T*, T**
    eff: Dict[int, float] = dataclasses.field(default_factory=dict)  # non-unit efficiencies


@dataclasses.dataclass
class Mechanism:
    name: str
    elements: List[str]
    species: List[str]
    comp: np.ndarray               # [K, n_elem] int
    W: np.ndarray                  # [K] kg/mol
    Tlow: np.ndarray               # [K]
    Tmid: np.ndarray
    Thigh: np.ndarray
    a_low: np.ndarray              # [K, 7]
    a_high: np.ndarray             # [K, 7]
    reactions: List[Reaction]
    inert: List[int]

    @property
    def K(self) -> int:
        return len(self.species)

    @property
    def R(self) -> int:
        return len(self.reactions)


@dataclasses.dataclass(frozen=True)
class MechSpec:
    name: str
    seed: int
    n_species: int                 # including inerts
    n_reactions: int
    frac_three_body: float
    frac_troe: float
    n_three_body: Optional[int] = None   # exact counts override the fractions
    n_troe: Optional[int] = None
    max_c: int = 3
    max_h: int = 8
    max_o: int = 2
    inerts: Tuple[str, ...] = ("N2",)


# ---------------------------------------------------------------------------
# species sets
# ---------------------------------------------------------------------------

def _formula(c: Dict[str, int]) -> str:
    return "".join(f"{e}{c[e] if c[e] > 1 else ''}" for e in ("C", "H", "O", "N", "Ar") if c.get(e, 0))


def _species_set(spec: MechSpec, rng: np.random.Generator) -> List[Tuple[str, Dict[str, int]]]:
    if spec.n_species == 13:
        return list(M13_SPECIES)
    base = [s for s in M13_SPECIES if s[0] != "N2"]
    have = {_formula(c) for _, c in base}
    pool = []
    for x in range(spec.max_c + 1):
        for y in range(spec.max_h + 1):
            for z in range(spec.max_o + 1):
                if x + y + z == 0:
                    continue
                c = {k: v for k, v in (("C", x), ("H", y), ("O", z)) if v}
                if _formula(c) in have:
                    continue
                if x == 1 and y == 0 and z == 0:
                    continue  # bare C atom left out
                pool.append(c)
    need = spec.n_species - len(base) - len(spec.inerts)
    pick = rng.choice(len(pool), size=need, replace=False)
    out = list(base) + [(_formula(pool[i]), pool[i]) for i in sorted(pick)]
    inert_comp = {"N2": {"N": 2}, "Ar": {"Ar": 1}}
    out += [(n, inert_comp[n]) for n in spec.inerts]
    return out


# ---------------------------------------------------------------------------
# thermodynamics: a smooth c_p(T) model fitted by two NASA-7 ranges
# ---------------------------------------------------------------------------

def _einstein(theta: np.ndarray, T: np.ndarray) -> np.ndarray:
    x = theta[None, :] / T[:, None]
    ex = np.exp(-x)
    return (x * x * ex / (1.0 - ex) ** 2).sum(axis=1)


def _cp_model(natoms: int, thetas: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Dimensionless c_p/R of an ideal gas with Einstein vibrational modes."""
    if natoms == 1:
        return np.full_like(T, 2.5)
    if natoms == 2:
        return 3.5 + _einstein(thetas, T)
    return 4.0 + _einstein(thetas, T)


def _fit_nasa7(cp_fn, hf298: float, s298: float, Tlow=300.0, Tmid=1000.0, Thigh=6000.0):
    """Fit a_1..a_5 on both ranges (c_p continuous at Tmid), then a_6, a_7 so that
    h(298.15) = hf298, s(298.15) = s298 and h, s are continuous at Tmid."""
    tl = np.linspace(Tlow, Tmid, 60)
    th = np.linspace(Tmid, Thigh, 80)
    Al = np.vander(tl / 1000.0, 5, increasing=True)
    Ah = np.vander(th / 1000.0, 5, increasing=True)
    bl = cp_fn(tl)
    bh = cp_fn(th)
    # KKT for min |Al cl - bl|^2 + |Ah ch - bh|^2  s.t.  pl(1) - ph(1) = 0
    n = 10
    M = np.zeros((n + 1, n + 1))
    rhs = np.zeros(n + 1)
    M[:5, :5] = 2 * Al.T @ Al
    M[5:10, 5:10] = 2 * Ah.T @ Ah
    g = np.concatenate([np.ones(5), -np.ones(5)])  # value at tau = 1
    M[:10, 10] = g
    M[10, :10] = g
    rhs[:5] = 2 * Al.T @ bl
    rhs[5:10] = 2 * Ah.T @ bh
    sol = np.linalg.solve(M, rhs)
    if np.ptp(bl) == 0.0 and np.ptp(bh) == 0.0 and bl[0] == bh[0]:
        sol = np.zeros(10)          # constant c_p (monatomic): exact coefficients
        sol[0] = sol[5] = bl[0]
    scale = np.array([1.0, 1e-3, 1e-6, 1e-9, 1e-12])
    al = np.zeros(7)
    ah = np.zeros(7)
    al[:5] = sol[:5] * scale
    ah[:5] = sol[5:10] * scale

    def hpoly(a, T):   # integral of c_p/R dT without the constant
        return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5

    def spoly(a, T):   # integral of c_p/(R T) dT without the constant
        return a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4

    T0 = 298.15
    al[5] = hf298 / R_U - hpoly(al, T0)
    al[6] = s298 / R_U - spoly(al, T0)
    ah[5] = hpoly(al, Tmid) + al[5] - hpoly(ah, Tmid)
    ah[6] = spoly(al, Tmid) + al[6] - spoly(ah, Tmid)
    return al, ah


# ---------------------------------------------------------------------------
# reactions
# ---------------------------------------------------------------------------

def _candidates(comp: np.ndarray, active: Sequence[int]):
    """Element-balanced candidates with 1-2 species per side.
    Returns (dissociation list [(AB,), (A,B)], exchange-by-composition dict)."""
    singles = {}
    for a in active:
        singles.setdefault(tuple(comp[a]), []).append(a)
    pairs: Dict[tuple, List[Tuple[int, int]]] = {}
    for i, a in enumerate(active):
        for b in active[i:]:
            key = tuple(comp[a] + comp[b])
            pairs.setdefault(key, []).append((a, b))
    dissoc = []
    for key, lst in pairs.items():
        for ab in singles.get(key, []):
            for p in lst:
                if ab in p:
                    continue
                dissoc.append(((ab,), p))
    exch_keys = [k for k, v in pairs.items() if len(v) >= 2]
    return dissoc, pairs, exch_keys


def _draw_arrhenius(rng: np.random.Generator, order: int):
    A_cgs = 10.0 ** rng.uniform(6.0, 14.0)
    b = rng.uniform(-1.5, 2.0)
    Ea = rng.uniform(0.0, 40.0) * 1000.0 * CAL
    return A_cgs * (1e-6) ** (order - 1), b, Ea


def make_mechanism(spec: MechSpec) -> Mechanism:
    rng = np.random.default_rng(spec.seed)
    sp = _species_set(spec, rng)
    elements = sorted({e for _, c in sp for e in c}, key=lambda e: ["H", "O", "C", "N", "Ar"].index(e))
    K = len(sp)
    comp = np.array([[c.get(e, 0) for e in elements] for _, c in sp], dtype=np.int64)
    W = np.array([sum(ATOMIC_WEIGHT[e] * n for e, n in c.items()) for _, c in sp]) * 1e-3
    names = [n for n, _ in sp]
    inert = [names.index(n) for n in spec.inerts]

    # thermo
    a_low = np.zeros((K, 7))
    a_high = np.zeros((K, 7))
    hf = np.zeros(K)
    for k, (name, c) in enumerate(sp):
        natoms = sum(c.values())
        nmodes = 1 if natoms == 2 else max(0, 3 * natoms - 6)
        thetas = np.exp(rng.uniform(math.log(400.0), math.log(4500.0), size=nmodes))
        hf[k] = 0.0 if name in ELEMENT_REFERENCE else rng.uniform(-HF_RANGE, HF_RANGE)
        s298 = 110.0 + 25.0 * (natoms - 1) + rng.uniform(0.0, 40.0)
        a_low[k], a_high[k] = _fit_nasa7(lambda T, n=natoms, th=thetas: _cp_model(n, th, T), hf[k], s298)

    active = [k for k in range(K) if k not in inert]
    dissoc, pairs, exch_keys = _candidates(comp, active)
    n3 = spec.n_three_body if spec.n_three_body is not None else int(round(spec.frac_three_body * spec.n_reactions))
    nt = spec.n_troe if spec.n_troe is not None else int(round(spec.frac_troe * spec.n_reactions))
    ne = spec.n_reactions - n3 - nt
    if n3 + nt > len(dissoc):
        raise ValueError("not enough dissociation candidates")

    for attempt in range(200):
        used = set()
        chosen: List[Tuple[int, tuple, tuple]] = []
        order_d = rng.permutation(len(dissoc))
        for idx in order_d:
            if len(chosen) >= n3 + nt:
                break
            l, r = dissoc[idx]
            key = frozenset([l, r])
            if key in used:
                continue
            used.add(key)
            chosen.append((THREE_BODY if len(chosen) < n3 else TROE, l, r))
        n_ex = 0
        tries = 0
        while n_ex < ne and tries < 100000:
            tries += 1
            key = exch_keys[rng.integers(len(exch_keys))]
            lst = pairs[key]
            i, j = rng.choice(len(lst), size=2, replace=False)
            l, r = lst[i], lst[j]
            if set(l) & set(r):
                continue
            kk = frozenset([l, r])
            if kk in used:
                continue
            used.add(kk)
            chosen.append((ELEMENTARY, l, r))
            n_ex += 1
        if n_ex < ne:
            raise ValueError("not enough exchange candidates")
        covered = {s for _, l, r in chosen for s in (*l, *r)}
        if covered >= set(active):
            break
    else:
        raise ValueError("could not cover every active species")

    reactions = []
    for kind, l, r in chosen:
        dH = sum(hf[s] for s in r) - sum(hf[s] for s in l)
        if dH > 0:       # write every reaction in its exothermic direction
            l, r = r, l
        order = len(l) + (1 if kind == THREE_BODY else 0)
        A, b, Ea = _draw_arrhenius(rng, order)
        rx = Reaction(kind, tuple(int(s) for s in l), tuple(int(s) for s in r), A, b, Ea)
        if kind == TROE:
            rx.A0 = A * 10.0 ** rng.uniform(3.0, 7.0) * 1e-6
            rx.b0, rx.Ea0 = b, Ea
            rx.troe = (rng.uniform(0.3, 0.9),
                       math.exp(rng.uniform(math.log(10.0), math.log(1000.0))),
                       math.exp(rng.uniform(math.log(500.0), math.log(5000.0))),
                       math.exp(rng.uniform(math.log(1000.0), math.log(10000.0))))
        if kind in (THREE_BODY, TROE):
            for k in range(K):
                if rng.uniform() < 0.25:
                    rx.eff[k] = rng.uniform(0.4, 6.0)
        reactions.append(rx)

    return Mechanism(spec.name, elements, names, comp, W,
                     np.full(K, 300.0), np.full(K, 1000.0), np.full(K, 6000.0),
                     a_low, a_high, reactions, inert)


# ---------------------------------------------------------------------------
# file format
# ---------------------------------------------------------------------------

def mech_text(m: Mechanism) -> str:
    """Serialise a mechanism.  Whitespace-separated tokens, '#' starts a comment.

        rkmech 1
        name <str>
        elements <E> <sym>...
        species <K>
          <name> <W kg/mol> <count per element...>          (K lines)
        thermo
          <k> <Tlow> <Tmid> <Thigh> <a_low 1..7> <a_high 1..7>  (K lines)
        reactions <R>
          <kind> <nr> <reac...> <np> <prod...> <A> <b> <Ea>
                 [kind 2: <A0> <b0> <Ea0> <a> <T***> <T*> <T**>]
                 [kind 1,2: <neff> (<k> <alpha>)...]
        end

    kind 0 elementary, 1 third-body, 2 Troe falloff.  Units SI: A in
    (m^3/mol)^(order-1)/s where order counts reactant slots (+1 for the third
    body of kind 1; A0 of kind 2 has order+1), Ea in J/mol.  Efficiencies not
    listed are 1.  All reactions are reversible.
    """
    f = lambda x: repr(float(x))
    out = ["rkmech 1", f"name {m.name}", "elements " + str(len(m.elements)) + " " + " ".join(m.elements),
           f"species {m.K}"]
    for k in range(m.K):
        out.append(f"{m.species[k]} {f(m.W[k])} " + " ".join(str(int(c)) for c in m.comp[k]))
    out.append("thermo")
    for k in range(m.K):
        out.append(" ".join([str(k), f(m.Tlow[k]), f(m.Tmid[k]), f(m.Thigh[k])]
                            + [f(a) for a in m.a_low[k]] + [f(a) for a in m.a_high[k]]))
    out.append(f"reactions {m.R}")
    for r in m.reactions:
        toks = [str(r.kind), str(len(r.reac))] + [str(s) for s in r.reac] + [str(len(r.prod))] + \
               [str(s) for s in r.prod] + [f(r.A), f(r.b), f(r.Ea)]
        if r.kind == TROE:
            toks += [f(r.A0), f(r.b0), f(r.Ea0)] + [f(x) for x in r.troe]
        if r.kind in (THREE_BODY, TROE):
            toks.append(str(len(r.eff)))
            for k in sorted(r.eff):
                toks += [str(k), f(r.eff[k])]
        out.append(" ".join(toks))
    out.append("end")
    return "\n".join(out) + "\n"


def write_mech(m: Mechanism, path: str) -> str:
    text = mech_text(m)
    with open(path, "w") as fh:
        fh.write(text)
    return path


# ---------------------------------------------------------------------------
# states (rows: T, Y_1..Y_K, P), returned as [n, K+2] float64
# ---------------------------------------------------------------------------

def uniform_states(K: int, n: int, seed: int, T_range=(900.0, 2200.0), P_atm=(1.0, 25.0), alpha=0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    T = rng.uniform(*T_range, size=n)
    P = P_ATM * np.exp(rng.uniform(math.log(P_atm[0]), math.log(P_atm[1]), size=n))
    Y = rng.dirichlet(np.full(K, alpha), size=n)
    Y /= Y.sum(axis=1, keepdims=True)
    return np.concatenate([T[:, None], Y, P[:, None]], axis=1)


def pasr_like_states(K: int, n: int, seed: int, templates: np.ndarray, frac_fresh=0.3,
                     fresh_T=(900.0, 1200.0), sigma=0.01) -> np.ndarray:
    """PaSR-like mix: `frac_fresh` fresh mixture (uniform T in `fresh_T`,
    log-uniform P in 1-25 atm, Dirichlet(0.5) composition) and the rest burnt,
    near-equilibrium states drawn from `templates` ([m, K+2] rows) with a
    per-species lognormal perturbation of the mass fractions, renormalised.
    Rows are shuffled with a seeded permutation so every wavefront mixes both."""
    rng = np.random.default_rng(seed)
    n_fresh = int(round(frac_fresh * n))
    fresh = uniform_states(K, n_fresh, int(rng.integers(1 << 31)), T_range=fresh_T)
    n_burnt = n - n_fresh
    pick = rng.integers(len(templates), size=n_burnt)
    burnt = templates[pick].copy()
    Y = burnt[:, 1:K + 1] * np.exp(sigma * rng.standard_normal((n_burnt, K)))
    Y = np.clip(Y, 0.0, None)
    Y /= Y.sum(axis=1, keepdims=True)
    burnt[:, 1:K + 1] = Y
    out = np.concatenate([fresh, burnt], axis=0)
    return out[rng.permutation(n)]


def template_seed_states(K: int, n: int, seed: int) -> np.ndarray:
    """Starting points of the burnt templates: T uniform 1800-2400 K, P
    log-uniform 1-25 atm, Dirichlet(0.5) composition (relaxed at fixed T, P
    by a separate step before use)."""
    return uniform_states(K, n, seed, T_range=(1800.0, 2400.0))


def to_soa(states: np.ndarray) -> np.ndarray:
    """[n, K+2] rows -> contiguous SoA [(K+2), n] (component-major)."""
    return np.ascontiguousarray(states.T)
