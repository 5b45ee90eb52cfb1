"""Workload definitions: synthetic mechanisms and state sets.

Mechanism sizes follow the paper's two models (13 species / 27 reversible
reactions and 53 species / 325 reactions, Sec. 2.2) plus a 150-species one;
tolerances are the paper's atol = 1e-10, rtol = 1e-6 (Sec. 2.1); global steps
are 1e-6 s and 1e-4 s (Sec. 3).
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional, Tuple

import numpy as np

from . import gen

ATOL = 1e-10
RTOL = 1e-6
DT_SMALL = 1e-6
DT_LARGE = 1e-4

MECHS = {
    "M13": gen.MechSpec("M13", seed=13027, n_species=13, n_reactions=27, frac_three_body=0.0,
                        frac_troe=0.0, n_three_body=4, n_troe=2),
    "M53": gen.MechSpec("M53", seed=53325, n_species=53, n_reactions=325, frac_three_body=0.15,
                        frac_troe=0.08, inerts=("N2", "Ar")),
    "M150": gen.MechSpec("M150", seed=1501000, n_species=150, n_reactions=1000, frac_three_body=0.15,
                         frac_troe=0.10, max_c=7, max_h=16, inerts=("N2", "Ar")),
}

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    mech: str
    n_states: int
    dts: Tuple[float, ...]
    states: str            # "uniform" or "pasr"
    seed: int


WORKLOADS = {
    "cfg0": Workload("cfg0", "M13", 4096, (DT_SMALL,), "uniform", 1000),
    "cfg1": Workload("cfg1", "M13", 262144, (DT_SMALL, DT_LARGE), "pasr", 1001),
    "cfg2": Workload("cfg2", "M53", 131072, (DT_SMALL, DT_LARGE), "pasr", 1002),
    # the 53-species states of cfg2 with the learned predictor
    "cfg3": Workload("cfg3", "M53", 131072, (DT_SMALL, DT_LARGE), "pasr", 1002),
    "cfg4": Workload("cfg4", "M150", 65536, (DT_LARGE,), "pasr", 1004),
}

TEMPLATE_SEEDS = {"M13": 2013, "M53": 2053, "M150": 2150}
N_TEMPLATES = 1024


def mech_path(name: str, directory: Optional[str] = None) -> str:
    """Write (once) and return the path of a synthetic mechanism file."""
    directory = directory or DATA_DIR
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, f"{name}.mech")
    text = gen.mech_text(gen.make_mechanism(MECHS[name]))
    if not os.path.exists(path) or open(path).read() != text:
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            fh.write(text)
        os.replace(tmp, path)
    return path


def template_path(mech: str) -> str:
    return os.path.join(DATA_DIR, f"{mech}_burnt_templates.npy")


def load_templates(mech: str) -> np.ndarray:
    return np.load(template_path(mech), allow_pickle=False)


def states_for(wl: Workload, n: Optional[int] = None) -> np.ndarray:
    """[n, K+2] rows for a workload (first n of the full seeded set)."""
    K = MECHS[wl.mech].n_species
    if wl.states == "uniform":
        s = gen.uniform_states(K, wl.n_states, wl.seed)
    else:
        s = gen.pasr_like_states(K, wl.n_states, wl.seed, load_templates(wl.mech))
    return s if n is None else s[:n]
