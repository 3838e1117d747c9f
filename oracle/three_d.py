"""Three-dimensional Poisson problem with the hybrid Schwarz / p-multigrid
method: the extension the paper names in its conclusions (Section 5), built
from the same ingredients as the 2-D path.

Test infrastructure (the oracle): plain NumPy/SciPy FP64, no fast
diagonalisation, no blocking.  Node arrays are U[z][y][x] (x fastest) with the
Dirichlet boundary nodes kept and zero.

* Operator (Section 2, tensor-product form, extended to three directions):
      A = M_z (x) M_y (x) L_x + M_z (x) L_y (x) M_x + L_z (x) M_y (x) M_x,
  applied as three 1-D products along the axes.
* Subdomains (Section 3.1): the products of the 1-D extended-element windows;
  the local problem is the principal submatrix of A, solved densely; the 1-D
  weights multiply (w_z w_y w_x), so the partition of unity carries over.
* Transfers (Section 3.2): the 1-D interpolation along each axis; the
  restriction is its transpose.  Coarse solve: sparse LU of A_0.
* Algorithm 3 (V-cycle) and Algorithm 4 (MGCG, oracle.mgcg) unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .discretization import DIRICHLET, Axis
from .multigrid import level_orders, level_overlap, prolongation_1d
from .schwarz import Subdomain1D


def _along(M, U, axis):
    """Apply the matrix M along one axis of the 3-D array U."""
    return np.moveaxis(np.tensordot(M, np.moveaxis(U, axis, 0), axes=(1, 0)), 0, axis)


class Space3:
    """Tensor-product SEM space on one level (Dirichlet)."""

    def __init__(self, xb, yb, zb, p: int):
        self.p = p
        self.bc = DIRICHLET
        self.ax, self.ay, self.az = Axis(xb, p, DIRICHLET), Axis(yb, p, DIRICHLET), Axis(zb, p, DIRICHLET)
        self.Lx, self.Mx = self.ax.assemble()
        self.Ly, self.My = self.ay.assemble()
        self.Lz, self.Mz = self.az.assemble()
        self.shape = (self.az.N, self.ay.N, self.ax.N)
        self.mask = (self.az.unknown_mask()[:, None, None] & self.ay.unknown_mask()[None, :, None]
                     & self.ax.unknown_mask()[None, None, :])

    def zero_boundary(self, U):
        return np.where(self.mask, U, 0.0)

    def coords(self):
        return self.ax.coords(), self.ay.coords(), self.az.coords()

    def apply_A(self, U):
        U = self.zero_boundary(U)
        out = _along(self.Mz, _along(self.My, _along(self.Lx, U, 2), 1), 0)
        out += _along(self.Mz, _along(self.Ly, _along(self.Mx, U, 2), 1), 0)
        out += _along(self.Lz, _along(self.My, _along(self.Mx, U, 2), 1), 0)
        return self.zero_boundary(out)

    def mass(self, F):
        m = (np.diag(self.Mz)[:, None, None] * np.diag(self.My)[None, :, None]
             * np.diag(self.Mx)[None, None, :])
        return self.zero_boundary(m * F)

    def dense_A(self):
        """A on the unknowns by Kronecker products (z slowest, x fastest)."""
        mx, my, mz = self.ax.unknown_mask(), self.ay.unknown_mask(), self.az.unknown_mask()
        Lx, Mx = self.Lx[np.ix_(mx, mx)], self.Mx[np.ix_(mx, mx)]
        Ly, My = self.Ly[np.ix_(my, my)], self.My[np.ix_(my, my)]
        Lz, Mz = self.Lz[np.ix_(mz, mz)], self.Mz[np.ix_(mz, mz)]
        return (np.kron(Mz, np.kron(My, Lx)) + np.kron(Mz, np.kron(Ly, Mx))
                + np.kron(Lz, np.kron(My, Mx)))


class SchwarzLevel3:
    """Weighted additive Schwarz (Algorithm 2) on one 3-D level: one extended
    element per subdomain, dense local inverses grouped by type triple."""

    def __init__(self, space: Space3, n_o: int, wf: int = 5):
        self.space = space
        self.n_o = n_o
        self.wf = wf
        ax, ay, az = space.ax, space.ay, space.az
        self.sx = [Subdomain1D(ax, space.Lx, space.Mx, e, n_o) for e in range(ax.n)]
        self.sy = [Subdomain1D(ay, space.Ly, space.My, e, n_o) for e in range(ay.n)]
        self.sz = [Subdomain1D(az, space.Lz, space.Mz, e, n_o) for e in range(az.n)]
        self.inv = {}
        for sz in self.sz:
            for sy in self.sy:
                for sx in self.sx:
                    k = (sz.key(), sy.key(), sx.key())
                    if k not in self.inv:
                        self.inv[k] = np.linalg.inv(local_matrix3(sz, sy, sx))

    def weights(self, ez, ey, ex):
        wz = self.sz[ez].weights(self.wf)
        wy = self.sy[ey].weights(self.wf)
        wx = self.sx[ex].weights(self.wf)
        return wz[:, None, None] * wy[None, :, None] * wx[None, None, :]

    def corrections(self, R):
        dU = np.zeros(self.space.shape)
        for ez, sz in enumerate(self.sz):
            for ey, sy in enumerate(self.sy):
                for ex, sx in enumerate(self.sx):
                    idx = np.ix_(sz.glob, sy.glob, sx.glob)
                    Rs = R[idx]
                    d = (self.inv[(sz.key(), sy.key(), sx.key())] @ Rs.ravel()).reshape(Rs.shape)
                    dU[idx] += self.weights(ez, ey, ex) * d
        return dU

    def smooth(self, U, F, n_it: int):
        sp = self.space
        for _ in range(n_it):
            R = sp.zero_boundary(F - sp.apply_A(U))
            U = U + self.corrections(R)
        return U


def local_matrix3(sz, sy, sx):
    """A_ss = M_z (x) M_y (x) L_x + M_z (x) L_y (x) M_x + L_z (x) M_y (x) M_x
    on the subdomain's unknowns (z slowest)."""
    return (np.kron(sz.Ms, np.kron(sy.Ms, sx.Ls)) + np.kron(sz.Ms, np.kron(sy.Ls, sx.Ms))
            + np.kron(sz.Ls, np.kron(sy.Ms, sx.Ms)))


def fdm_solve3(sz, sy, sx, Rs):
    """Fast diagonalisation in three directions (the GPU's method), kept to be
    checked against the dense local inverse:
    A_ss^{-1} = (S_z (x) S_y (x) S_x) (Lz + Ly + Lx)^{-1} (S_z (x) S_y (x) S_x)^T."""
    from .schwarz import fdm_factors
    Sx, lx = fdm_factors(sx.Ls, sx.Ms)
    Sy, ly = fdm_factors(sy.Ls, sy.Ms)
    Sz, lz = fdm_factors(sz.Ls, sz.Ms)
    T = _along(Sz.T, _along(Sy.T, _along(Sx.T, Rs, 2), 1), 0)
    T = T / (lz[:, None, None] + ly[None, :, None] + lx[None, None, :])
    return _along(Sz, _along(Sy, _along(Sx, T, 2), 1), 0)


class Multigrid3:
    """p-multigrid hierarchy p_{l-1} = ceil(p_l / 2) in 3-D (Poisson, Dirichlet)."""

    def __init__(self, xb, yb, zb, p: int, overlap_rule: int = 0, n_o: int = 1, wf: int = 5):
        self.orders = level_orders(p)
        self.L = len(self.orders) - 1
        self.bc = DIRICHLET
        self.spaces = [Space3(xb, yb, zb, q) for q in self.orders]
        self.overlaps = [0] + [level_overlap(overlap_rule, n_o, q) for q in self.orders[1:]]
        self.P = [None] + [
            tuple(prolongation_1d(getattr(self.spaces[l - 1], a), getattr(self.spaces[l], a))
                  for a in ("ax", "ay", "az"))
            for l in range(1, self.L + 1)]
        self.schwarz = [None] + [SchwarzLevel3(self.spaces[l], self.overlaps[l], wf)
                                 for l in range(1, self.L + 1)]
        s0 = self.spaces[0]
        self.A0_lu = spla.splu(sps.csc_matrix(s0.dense_A()))

    def op(self, l: int, U):
        return self.spaces[l].apply_A(U)

    def residual(self, l: int, U, F):
        return self.spaces[l].zero_boundary(F - self.op(l, U))

    def prolong(self, l: int, Uc):
        Px, Py, Pz = self.P[l]
        return self.spaces[l].zero_boundary(_along(Pz, _along(Py, _along(Px, Uc, 2), 1), 0))

    def restrict(self, l: int, R):
        Px, Py, Pz = self.P[l]
        return self.spaces[l - 1].zero_boundary(_along(Pz.T, _along(Py.T, _along(Px.T, R, 2), 1), 0))

    def smooth(self, l: int, U, F, n_it: int):
        return U if n_it == 0 else self.schwarz[l].smooth(U, F, n_it)

    def coarse_solve(self, F0):
        s = self.spaces[0]
        U = np.zeros(s.shape)
        U[s.mask] = self.A0_lu.solve(F0[s.mask])
        return U

    def vcycle(self, U, F, ns1=None, ns2=None):
        """Algorithm 3 with u_{l-1} = 0 (reading C-L3)."""
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
