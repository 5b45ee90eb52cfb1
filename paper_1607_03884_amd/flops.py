"""Algorithmic operation counts of the Radau IIA hot path.

Counts follow the formulas the kernels evaluate (add, sub, mul, div = 1 flop,
fused multiply-add = 2); every exp/log/pow/exp10 is one transcendental,
counted as 1 flop and also reported separately.  Per-state counters from the
integrator (f-evaluations, Jacobians, LU factorisations, Newton iterations,
step attempts) turn them into flops per launch.

With K species, N = K + 1 unknowns, R reactions of which R3 third-body and
RT Troe falloff:
  source terms  c_f = 38 K + 8 + 23 R + R3 (2K + 1) + RT (2K + 27)
                t_f = 3 + 2 R + 6 RT
  Jacobian      c_J = 58 K + 101 R + (R3 + RT) 10 K + 67 RT + 6 K^2
                t_J = 3 + 2 R + 6 RT
  LU of E1 (real) and E2 (complex)      (2/3 + 8/3) N^3 = 10/3 N^3
  Newton iteration: one real and one complex solve (2 N^2 + 8 N^2) plus the
    stage transformations and norm, 10 N^2 + 64 N
  error estimate: one real solve and the weighted norm, 2 N^2 + 8 N
  step bookkeeping (starting values, transformation, update) 48 N
"""
from __future__ import annotations

from dataclasses import dataclass

from . import gen


@dataclass(frozen=True)
class Costs:
    K: int
    N: int
    c_f: float
    t_f: float
    c_J: float
    t_J: float

    @classmethod
    def of(cls, mech: gen.Mechanism) -> "Costs":
        K, R = mech.K, mech.R
        R3 = sum(1 for r in mech.reactions if r.kind == gen.THREE_BODY)
        RT = sum(1 for r in mech.reactions if r.kind == gen.TROE)
        c_f = 38 * K + 8 + 23 * R + R3 * (2 * K + 1) + RT * (2 * K + 27)
        t_f = 3 + 2 * R + 6 * RT
        c_J = 58 * K + 101 * R + (R3 + RT) * 10 * K + 67 * RT + 6 * K * K
        return cls(K, K + 1, float(c_f), float(t_f), float(c_J), float(t_f))

    def flops(self, st: dict) -> dict:
        """st: totals from stats_get (f_evals, jac_evals, lu_factor,
        newton_iters, steps, newton_fail)."""
        N = self.N
        fl = (st["f_evals"] * self.c_f + st["jac_evals"] * self.c_J
              + st["lu_factor"] * (10.0 / 3.0 * N ** 3 + N)
              + st["newton_iters"] * (10.0 * N * N + 64 * N)
              + (st["steps"] - st["newton_fail"]) * (2.0 * N * N + 8 * N)
              + st["steps"] * 48.0 * N)
        tr = st["f_evals"] * self.t_f + st["jac_evals"] * self.t_J
        return {"flops": float(fl), "transcendentals": float(tr)}
