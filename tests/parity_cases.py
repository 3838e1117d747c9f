"""Shared set-up for the GPU parity tests: the same problem built once in the
oracle and once in the HIP library, from the seeded generators."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from paper_1512_02390_amd import workloads as W

D, P = W.BC_DIRICHLET, W.BC_PERIODIC
FIXED, CEIL8, FLOOR8, CEIL2 = 0, 1, 2, 3
TOPHAT, ARITH, MULT = -1, -2, -3


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
    alpha_seed: int | None = None   # random width scales per grid line in [0.2, 1]
    elem_seed: int | None = None    # random per-element (alpha_e, rho_e)
    separable: bool = False         # separable local coefficients (variable nu)
    strong_nu: bool = False         # nu field with length 0.2 and sigma 1

    def breaks(self):
        if self.stretched:
            xb = W.geometric_breaks(self.nx, 1.0 / self.ny, 4.0)
        else:
            xb = W.uniform_breaks(self.nx, 1.3)
        yb = W.uniform_breaks(self.ny, 1.0)
        return xb, yb

    def alphas(self):
        """(alpha_x, alpha_y) per grid line, or (None, None) for the paper's
        weights.  Periodic: the last line is the first one, so it repeats it."""
        if self.alpha_seed is None:
            return None, None
        g = W.rng(self.alpha_seed)
        ax = g.uniform(0.2, 1.0, self.nx + 1)
        ay = g.uniform(0.2, 1.0, self.ny + 1)
        if self.bc == W.BC_PERIODIC:
            ax[-1], ay[-1] = ax[0], ay[0]
        return ax, ay

    def elem_params(self):
        """(n_e, 2) per-element (alpha_e, rho_e), e = ey * nx + ex, rounded to
        FP32 as the library receives them; or None."""
        if self.elem_seed is None:
            return None
        g = W.rng(self.elem_seed)
        a = g.uniform(0.2, 1.0, self.nx * self.ny)
        r = g.uniform(0.0, 0.5, self.nx * self.ny)
        return np.stack([a, r], axis=1).astype(np.float32).astype(np.float64)


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
    # width scales alpha != 1 per grid line (the hook of the learned parameters)
    Case("dir_p8_no2_alpha_stretch", 5, 4, 8, D, stretched=True, n_o=2, alpha_seed=11),
    Case("per_p6_no2_alpha", 4, 5, 6, P, n_o=2, alpha_seed=12),
    Case("dir_p12_ceil8_alpha_varnu", 3, 4, 12, D, stretched=True, rule=CEIL8, varnu=True,
         alpha_seed=13),
    # the seventh-order weight function of Table 1
    Case("per_p4_no1_septic", 4, 3, 4, P, wf=7),
    Case("dir_p16_ceil8_septic", 3, 2, 16, D, rule=CEIL8, wf=7),
    # per-element overlaps and widths with Shepard normalisation
    Case("dir_p8_elem_stretch", 5, 4, 8, D, stretched=True, elem_seed=21),
    Case("per_p6_elem_cubic", 4, 5, 6, P, wf=3, elem_seed=22),
    Case("dir_p12_elem_varnu_stretch", 3, 4, 12, D, stretched=True, varnu=True, elem_seed=23),
    Case("dir_p16_elem_arith", 3, 3, 16, D, wf=ARITH, elem_seed=24),
    Case("dir_p32_elem", 2, 2, 32, D, elem_seed=25),
    # wide FP64 tiles (m = 41) on meshes with several elements per type pair
    Case("per_p32_ceil8_varnu_wide", 4, 4, 32, P, rule=CEIL8, varnu=True),
    Case("dir_p32_ceil8_wide", 5, 2, 32, D, rule=CEIL8),
    # separable local coefficients per subdomain (variable nu)
    Case("dir_p8_sep_stretch", 5, 4, 8, D, stretched=True, rule=CEIL8, varnu=True,
         separable=True),
    Case("per_p6_sep_no2_strong", 4, 4, 6, P, n_o=2, varnu=True, separable=True, strong_nu=True),
    Case("dir_p16_sep_strong", 3, 3, 16, D, rule=CEIL8, varnu=True, separable=True,
         strong_nu=True),
    Case("dir_p12_sep_no0", 4, 3, 12, D, n_o=0, varnu=True, separable=True),
    # multiplicative Schwarz (Algorithm 1): sequential sweeps, Poisson
    Case("dir_p4_mult", 5, 4, 4, D, n_o=1, wf=MULT),
    Case("per_p6_mult_no2", 4, 3, 6, P, n_o=2, wf=MULT),
    Case("dir_p8_mult_ceil8_stretch", 4, 3, 8, D, stretched=True, rule=CEIL8, wf=MULT),
    Case("dir_p16_mult_no0", 3, 2, 16, D, n_o=0, wf=MULT),
]


def nu_field(case: Case):
    if not case.varnu:
        return None
    if case.strong_nu:
        return W.GaussianFieldNu(seed=W.SEED_GRF, ell=0.2, sigma=1.0)
    return W.GaussianFieldNu(seed=W.SEED_GRF, ell=0.5, sigma=0.3)


def build_oracle(case: Case):
    from oracle.discretization import Space
    from oracle.multigrid import Multigrid
    xb, yb = case.breaks()
    NU = None
    nu = nu_field(case)
    if nu is not None:
        top = Space(xb, yb, case.p, case.bc)
        NU = W.nodal(nu.nu, top.x(), top.y())
    ax, ay = case.alphas()
    ep = case.elem_params()
    if ep is not None:
        ep = (ep[:, 0].reshape(case.ny, case.nx), ep[:, 1].reshape(case.ny, case.nx))
    return Multigrid(xb, yb, case.p, case.bc, case.rule, case.n_o, case.wf, NU=NU,
                     alpha_x=ax, alpha_y=ay, overlaps=case.overlaps, elem_params=ep,
                     local_solve="separable" if case.separable else "mean"), NU


def build_gpu(case: Case, NU=None, precision=0):
    from paper_1512_02390_amd.sem import Solver
    xb, yb = case.breaks()
    ax, ay = case.alphas()
    from paper_1512_02390_amd.sem import LOCAL_MEAN, LOCAL_SEPARABLE
    return Solver(xb, yb, case.p, case.bc, case.rule, case.n_o, case.wf, nu=NU,
                  precision=precision, overlaps=case.overlaps, alpha_x=ax, alpha_y=ay,
                  elem_params=case.elem_params(),
                  local_solve=LOCAL_SEPARABLE if case.separable else LOCAL_MEAN)


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)
