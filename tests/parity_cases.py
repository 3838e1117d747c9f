"""Shared set-up for the GPU parity tests: the same problem built once in the
oracle and once in the HIP library, from the seeded generators."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from paper_1512_02390_amd import workloads as W

D, P = W.BC_DIRICHLET, W.BC_PERIODIC
FIXED, CEIL8, FLOOR8, CEIL2 = 0, 1, 2, 3
TOPHAT, ARITH = -1, -2


@dataclass(frozen=True)
class Case:
    name: str
    nx: int
    ny: int
    p: int
    bc: int
    stretched: bool = False
    rule: int = FIXED
    n_o: int = 1
    wf: int = 5
    varnu: bool = False
    overlaps: tuple | None = None   # explicit n_o per level (entry 0 unused)

    def breaks(self):
        if self.stretched:
            xb = W.geometric_breaks(self.nx, 1.0 / self.ny, 4.0)
        else:
            xb = W.uniform_breaks(self.nx, 1.3)
        yb = W.uniform_breaks(self.ny, 1.0)
        return xb, yb


CASES = [
    Case("dir_p4_no1", 5, 4, 4, D),
    Case("dir_p1", 6, 5, 1, D),
    Case("dir_p2_no1", 4, 3, 2, D),
    Case("dir_p8_no3_stretch", 4, 3, 8, D, stretched=True, n_o=3),
    Case("per_p6_no2_cubic", 4, 3, 6, P, n_o=2, wf=3),
    Case("dir_p16_ceil8", 3, 3, 16, D, rule=CEIL8),
    Case("dir_p12_ceil8_varnu_stretch", 4, 4, 12, D, stretched=True, rule=CEIL8, varnu=True),
    Case("per_p5_arith", 4, 4, 5, P, wf=ARITH),
    Case("dir_p32_ceil8", 2, 3, 32, D, rule=CEIL8),
    Case("dir_p3_no2_tophat", 7, 5, 3, D, n_o=2, wf=TOPHAT),
    Case("per_p8_varnu", 3, 4, 8, P, rule=CEIL8, varnu=True),
    Case("dir_p7_no6_linear_stretch", 3, 2, 7, D, stretched=True, n_o=6, wf=1),
    Case("dir_single_element_p9", 1, 1, 9, D, n_o=3),
    Case("dir_p12_ceil2_varnu_stretch", 4, 3, 12, D, stretched=True, rule=CEIL2, varnu=True),
    Case("dir_p32_levels_varnu_stretch", 2, 2, 32, D, stretched=True, varnu=True,
         overlaps=(0, 1, 1, 2, 4, 7)),
]


def nu_field(case: Case):
    return W.GaussianFieldNu(seed=W.SEED_GRF, ell=0.5, sigma=0.3) if case.varnu else None


def build_oracle(case: Case):
    from oracle.discretization import Space
    from oracle.multigrid import Multigrid
    xb, yb = case.breaks()
    NU = None
    nu = nu_field(case)
    if nu is not None:
        top = Space(xb, yb, case.p, case.bc)
        NU = W.nodal(nu.nu, top.x(), top.y())
    return Multigrid(xb, yb, case.p, case.bc, case.rule, case.n_o, case.wf, NU=NU,
                     overlaps=case.overlaps), NU


def build_gpu(case: Case, NU=None, precision=0):
    from paper_1512_02390_amd.sem import Solver
    xb, yb = case.breaks()
    return Solver(xb, yb, case.p, case.bc, case.rule, case.n_o, case.wf, nu=NU,
                  precision=precision, overlaps=case.overlaps)


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)
