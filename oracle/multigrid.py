"""p-multigrid V-cycle (Section 3.2, Algorithm 3).

Levels: p_L = p on top, p_{l-1} = ceil(p_l / 2) down to p_0 = 1.  For powers of
two this is the paper's p_l = 2^l; the ceiling is our reading for other p.
A_l is the same discretisation with elements of order p_l.  The correction is
carried from level l-1 to l by the embedded interpolation I_l (the coarse
element polynomial evaluated at the fine GLL nodes) and the residual is
restricted with its transpose.  The coarse problem is solved exactly with the
pseudoinverse A_0^+; for a singular (periodic) A_0 the right side is first
projected onto the range of A_0, i.e. its mean is removed, and the solution
returned has zero mean.

Overlap per level l > 0: fixed n_o, ceil(p_l/8), floor(p_l/8) or ceil(p_l/2)
(Section 4), always clamped to [0, p_l - 1].

Variable diffusion: nu is given at the finest nodes; each coarser level uses
the element-wise Lagrange interpolant of it at its own GLL nodes, and all
levels share the finest level's element means nu_bar.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .discretization import PERIODIC, Space, element_mean
from .gll import gll, lagrange_matrix
from .schwarz import (ElementwiseSchwarzLevel, MultiplicativeSchwarzLevel, SchwarzLevel,
                      SeparableSchwarzLevel)
from .weights import WF_MULT

OVERLAP_FIXED, OVERLAP_CEIL8, OVERLAP_FLOOR8, OVERLAP_CEIL2 = 0, 1, 2, 3


def level_orders(p: int):
    ps = [p]
    while ps[-1] > 1:
        ps.append(math.ceil(ps[-1] / 2))
    return ps[::-1]           # index l = 0 .. L


def level_overlap(rule: int, n_o: int, p_l: int) -> int:
    if rule == OVERLAP_FIXED:
        v = n_o
    elif rule == OVERLAP_CEIL8:
        v = math.ceil(p_l / 8)
    elif rule == OVERLAP_FLOOR8:
        v = p_l // 8
    elif rule == OVERLAP_CEIL2:
        v = math.ceil(p_l / 2)
    else:
        raise ValueError(rule)
    return max(0, min(v, p_l - 1))


MAX_TILE = 48   # widest subdomain p_l + 1 + 2 n_o the per-element rule produces


def element_overlap(rho: float, p_l: int) -> int:
    """Per-element overlap on level l from an overlap ratio rho (learned
    parameters): ceil(rho p_l) clamped to [1, p_l - 1] and to a subdomain
    width p_l + 1 + 2 n_o of at most MAX_TILE nodes."""
    v = math.ceil(rho * p_l - 1e-12)
    v = min(max(v, 1), p_l - 1, (MAX_TILE - p_l - 1) // 2)
    return max(v, 0)


def prolongation_1d(axis_c, axis_f) -> np.ndarray:
    """P[i_f, i_c] = l^c_{a_c}(xi^f_{a_f}) within each element (all nodes)."""
    E = lagrange_matrix(axis_c.xi, axis_f.xi)        # (p_f+1, p_c+1)
    P = np.zeros((axis_f.N, axis_c.N))
    for e in range(axis_f.n):
        for a in range(axis_f.p + 1):
            for c in range(axis_c.p + 1):
                P[axis_f.node_index(e, a), axis_c.node_index(e, c)] = E[a, c]
    return P


def interpolate_nodal(space_from: Space, space_to: Space, V) -> np.ndarray:
    """Element-wise Lagrange interpolation of a nodal field to other GLL nodes."""
    E = lagrange_matrix(space_from.ax.xi, space_to.ax.xi)
    out = np.zeros(space_to.shape)
    for ey in range(space_to.ay.n):
        for ex in range(space_to.ax.n):
            gy_f, gx_f = space_from.element_nodes(ey, ex)
            gy_t, gx_t = space_to.element_nodes(ey, ex)
            out[np.ix_(gy_t, gx_t)] = E @ V[np.ix_(gy_f, gx_f)] @ E.T
    return out


class Multigrid:
    def __init__(self, xb, yb, p: int, bc: int, overlap_rule: int = OVERLAP_FIXED,
                 n_o: int = 1, wf: int = 5, NU=None, alpha_x=None, alpha_y=None, overlaps=None,
                 elem_params=None, local_solve: str = "mean"):
        """overlaps: optional explicit n_o per level (index 0 unused).
        elem_params: optional (alpha_e, rho_e), two (ny, nx) arrays of per-
        element width scales and overlap ratios; every level l > 0 then uses
        ElementwiseSchwarzLevel with n_o,e = element_overlap(rho_e, p_l).
        local_solve: "mean" (Section 4: A_ss^{-1} / nu_bar_s) or "separable"
        (variable nu only: SeparableSchwarzLevel, nu fitted per subdomain as
        a(x) b(y) on the level's own nodal nu)."""
        self.orders = level_orders(p)
        self.L = len(self.orders) - 1
        self.bc = bc
        self.spaces = [Space(xb, yb, q, bc) for q in self.orders]
        if overlaps is not None:
            self.overlaps = [0] + [int(v) for v in overlaps[1:]]
        else:
            self.overlaps = [0] + [level_overlap(overlap_rule, n_o, q) for q in self.orders[1:]]
        self.P = [None] + [
            (sps.csr_matrix(prolongation_1d(self.spaces[l - 1].ax, self.spaces[l].ax)),
             sps.csr_matrix(prolongation_1d(self.spaces[l - 1].ay, self.spaces[l].ay)))
            for l in range(1, self.L + 1)]
        # variable diffusion: nu per level and element means from the top level
        self.NU = None
        self.nubar = None
        if NU is not None:
            top = self.spaces[-1]
            self.NU = [interpolate_nodal(top, s, NU) for s in self.spaces[:-1]] + [np.array(NU)]
            self.nubar = element_mean(top, NU)
        if elem_params is not None:
            alpha_e = np.asarray(elem_params[0], dtype=np.float64)
            rho_e = np.asarray(elem_params[1], dtype=np.float64)
            self.elem_no = [None]
            self.schwarz = [None]
            for l in range(1, self.L + 1):
                q = self.orders[l]
                no = np.vectorize(lambda r: element_overlap(r, q))(rho_e).astype(int)
                self.elem_no.append(no)
                self.overlaps[l] = int(no.max())
                self.schwarz.append(ElementwiseSchwarzLevel(self.spaces[l], no, alpha_e, wf))
        elif local_solve == "separable":
            if NU is None:
                raise ValueError("separable local solves need a variable nu")
            self.schwarz = [None] + [
                SeparableSchwarzLevel(self.spaces[l], self.overlaps[l], wf, self.NU[l])
                for l in range(1, self.L + 1)]
        elif local_solve != "mean":
            raise ValueError("local_solve must be 'mean' or 'separable'")
        elif wf == WF_MULT:
            self.schwarz = [None] + [MultiplicativeSchwarzLevel(self.spaces[l], self.overlaps[l])
                                     for l in range(1, self.L + 1)]
        else:
            self.schwarz = [None] + [
                SchwarzLevel(self.spaces[l], self.overlaps[l], wf, alpha_x, alpha_y)
                for l in range(1, self.L + 1)]
        self._coarse_setup()

    # -- operators ------------------------------------------------------------
    def op(self, l: int, U):
        s = self.spaces[l]
        return s.apply_A(U) if self.NU is None else s.apply_B(U, self.NU[l])

    def residual(self, l: int, U, F):
        return self.spaces[l].zero_boundary(F - self.op(l, U))

    def prolong(self, l: int, Uc):
        """I_l u_{l-1} = P_y U_c P_x^T."""
        Px, Py = self.P[l]
        return self.spaces[l].zero_boundary(Py @ (Px @ Uc.T).T)

    def restrict(self, l: int, R):
        """I_l^T r = P_y^T R P_x."""
        Px, Py = self.P[l]
        return self.spaces[l - 1].zero_boundary(Py.T @ (Px.T @ R.T).T)

    def smooth(self, l: int, U, F, n_it: int):
        if n_it == 0:
            return U
        nu = None if self.NU is None else self.NU[l]
        return self.schwarz[l].smooth(U, F, n_it, nu, self.nubar)

    # -- coarse grid ------------------------------------------------------------
    def _coarse_setup(self):
        """Factor A_0 once.  Dirichlet Poisson: sparse LU of the Kronecker form
        (size grows with the mesh); otherwise dense Cholesky of A_0 (+ c 1 1^T
        when periodic, which is SPD and leaves A_0^+ f unchanged on the range)."""
        s = self.spaces[0]
        self.A0_lu = None
        if self.NU is None and self.bc != PERIODIC:
            mx, my = s.ax.unknown_mask(), s.ay.unknown_mask()
            Lx = sps.csr_matrix(s.Lx[np.ix_(mx, mx)])
            Mx = sps.csr_matrix(s.Mx[np.ix_(mx, mx)])
            Ly = sps.csr_matrix(s.Ly[np.ix_(my, my)])
            My = sps.csr_matrix(s.My[np.ix_(my, my)])
            A0 = (sps.kron(My, Lx) + sps.kron(Ly, Mx)).tocsc()
            self.A0_lu = spla.splu(A0)
            return
        A0 = s.dense_A() if self.NU is None else s.dense_B(self.NU[0])
        if self.bc == PERIODIC:
            n = A0.shape[0]
            A0 = A0 + (np.trace(A0) / n ** 2) * np.ones((n, n))
        self.A0_factor = sla.cho_factor(A0)

    def coarse_solve(self, F0):
        """u_0 = A_0^+ f_0 (Algorithm 3, coarse grid solution)."""
        s = self.spaces[0]
        f = F0[s.mask]
        if self.bc == PERIODIC:
            f = f - f.mean()
        if self.A0_lu is not None:
            u = self.A0_lu.solve(f)
        else:
            u = sla.cho_solve(self.A0_factor, f)
        if self.bc == PERIODIC:
            u = u - u.mean()
        U = np.zeros(s.shape)
        U[s.mask] = u
        return U

    # -- cycle --------------------------------------------------------------------
    def vcycle(self, U, F, ns1=None, ns2=None):
        """Algorithm 3 (MultigridCycle).  ns1[l], ns2[l]: pre/post smoothing
        steps on level l = 1..L (index 0 unused); default MG(1,0)."""
        L = self.L
        ns1 = [1] * (L + 1) if ns1 is None else ns1
        ns2 = [0] * (L + 1) if ns2 is None else ns2
        u = [None] * (L + 1)
        f = [None] * (L + 1)
        u[L], f[L] = np.array(U, dtype=np.float64), np.array(F, dtype=np.float64)
        for l in range(L, 0, -1):
            u[l] = self.smooth(l, u[l], f[l], ns1[l])
            f[l - 1] = self.restrict(l, self.residual(l, u[l], f[l]))
            u[l - 1] = np.zeros(self.spaces[l - 1].shape)
        u[0] = self.coarse_solve(f[0])
        for l in range(1, L + 1):
            u[l] = u[l] + self.prolong(l, u[l - 1])
            u[l] = self.smooth(l, u[l], f[l], ns2[l])
        return u[L]


def smoothing_schedule(L: int, kind: str = "mg10"):
    """(ns1, ns2) per level.  'mg10': one pre-smoothing; 'mg11': one pre and
    one post; 'var11': variable V-cycle with 2^(L-l) steps each (Section 4)."""
    if kind == "mg10":
        return [1] * (L + 1), [0] * (L + 1)
    if kind == "mg11":
        return [1] * (L + 1), [1] * (L + 1)
    if kind == "var11":
        s = [2 ** (L - l) for l in range(L + 1)]
        return s, list(s)
    raise ValueError(kind)
