"""Write the burnt near-equilibrium templates of the PaSR-like state mix.

The paper's PaSR databases are mostly near-equilibrium burnt particles plus
fresh inflow (Sec. 2.2).  The synthetic stand-in draws burnt states from
templates made here: seeded starting points (T uniform 1800-2400 K, P
log-uniform 1-25 atm, Dirichlet(0.5) composition) relaxed at fixed T and P
for 1 ms by this oracle's Radau IIA integrator, so that the composition sits
near the mechanism's equilibrium at that temperature.

Run:  python -m oracle.make_burnt_templates M13 [M53 M150]
Writes paper_1607_03884_amd/data/<mech>_burnt_templates.npy ([m, K+2] rows).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1607_03884_amd import configs, gen  # noqa: E402

RELAX_TIME = 1e-3


def make(name: str, n: int = configs.N_TEMPLATES, nthreads: int = 0) -> str:
    oracle.build()
    K = configs.MECHS[name].n_species
    m = oracle.Mech(configs.mech_path(name))
    start = gen.template_seed_states(K, n, configs.TEMPLATE_SEEDS[name])
    t0 = time.time()
    out, res = m.integrate(start, RELAX_TIME, opts=oracle.default_opts(isothermal=1), nthreads=nthreads)
    ok = res["status"] == 0
    if not ok.all():
        raise RuntimeError(f"{(~ok).sum()} template relaxations failed")
    out[:, 1:K + 1] = np.clip(out[:, 1:K + 1], 0.0, None)
    out[:, 1:K + 1] /= out[:, 1:K + 1].sum(axis=1, keepdims=True)
    path = configs.template_path(name)
    np.save(path, out)
    print(f"{name}: {n} templates in {time.time() - t0:.1f} s, median steps {np.median(res['nstep']):.0f} -> {path}")
    return path


if __name__ == "__main__":
    for name in sys.argv[1:] or ["M13"]:
        make(name)
