"""Spectral element discretisation on a Cartesian mesh (Section 2).

Node arrays are 2-D with rows along y and columns along x.  With Dirichlet
boundaries the array keeps the boundary nodes (always zero); with periodic
boundaries node n*p is node 0 and is not stored.

The global system matrix has the tensor-product form A = M_y (x) L_x +
L_y (x) M_x (Section 2, eq. system matrix), where M_* and L_* are the assembled
1-D mass and stiffness matrices.  With row-major vectorisation of a node array
U this is  A u = M_y U L_x^T + L_y U M_x^T.

The variable-coefficient operator B(nu) of Section 4 (eq. diffusion discrete
system) is built element by element with GLL quadrature; for nu = 1 it is the
same matrix as A, which the tests use as an independent check of both routes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sps

from .gll import gll, derivative_matrix, element_matrices

DIRICHLET = 0
PERIODIC = 1


@dataclass
class Axis:
    """One direction of the mesh at one polynomial order."""
    breaks: np.ndarray
    p: int
    bc: int

    def __post_init__(self):
        self.breaks = np.asarray(self.breaks, dtype=np.float64)
        self.n = len(self.breaks) - 1
        self.h = np.diff(self.breaks)
        self.xi, self.w = gll(self.p)
        self.N = self.n * self.p + (1 if self.bc == DIRICHLET else 0)

    def node_index(self, e: int, a: int) -> int:
        """Global node index of local node a of element e."""
        g = e * self.p + a
        return g % self.N if self.bc == PERIODIC else g

    def coords(self) -> np.ndarray:
        x = np.zeros(self.N)
        for e in range(self.n):
            for a in range(self.p + 1):
                if self.bc == PERIODIC and e * self.p + a == self.N:
                    continue        # the wrapped end node is node 0, at breaks[0]
                x[self.node_index(e, a)] = self.breaks[e] + 0.5 * self.h[e] * (self.xi[a] + 1.0)
        return x

    def unknown_mask(self) -> np.ndarray:
        m = np.ones(self.N, dtype=bool)
        if self.bc == DIRICHLET:
            m[0] = m[-1] = False
        return m

    def assemble(self):
        """Dense assembled 1-D stiffness L and (diagonal) mass M over all nodes.
        Element matrices: L^e = (2/h) L^, M^e = (h/2) W (Section 2)."""
        Lhat, What, _, _, _ = element_matrices(self.p)
        L = np.zeros((self.N, self.N))
        M = np.zeros((self.N, self.N))
        for e in range(self.n):
            idx = [self.node_index(e, a) for a in range(self.p + 1)]
            for a in range(self.p + 1):
                M[idx[a], idx[a]] += 0.5 * self.h[e] * What[a]
                for b in range(self.p + 1):
                    L[idx[a], idx[b]] += (2.0 / self.h[e]) * Lhat[a, b]
        return L, M


class Space:
    """Tensor-product SEM space on one multigrid level."""

    def __init__(self, xb, yb, p: int, bc: int):
        self.p = p
        self.bc = bc
        self.ax = Axis(xb, p, bc)
        self.ay = Axis(yb, p, bc)
        self.Lx, self.Mx = self.ax.assemble()
        self.Ly, self.My = self.ay.assemble()
        # the same matrices in sparse storage, used to apply the operator
        self._sLx, self._sMx = sps.csr_matrix(self.Lx), sps.csr_matrix(self.Mx)
        self._sLy, self._sMy = sps.csr_matrix(self.Ly), sps.csr_matrix(self.My)
        self.shape = (self.ay.N, self.ax.N)
        self.mask = self.ay.unknown_mask()[:, None] & self.ax.unknown_mask()[None, :]

    # -- helpers ------------------------------------------------------------
    def zero_boundary(self, U):
        return np.where(self.mask, U, 0.0)

    def x(self):
        return self.ax.coords()

    def y(self):
        return self.ay.coords()

    # -- operators ----------------------------------------------------------
    def apply_A(self, U):
        """A u = (M_y (x) L_x + L_y (x) M_x) u on the unknowns."""
        U = self.zero_boundary(U)
        # M_y U L_x^T + L_y U M_x^T, each product taken with the sparse factor
        t1 = self._sMy @ (self._sLx @ U.T).T
        t2 = self._sLy @ (self._sMx @ U.T).T
        return self.zero_boundary(t1 + t2)

    def mass(self, F):
        """(M_y (x) M_x) f for nodal values f: the discrete right-hand side."""
        return self.zero_boundary(np.diag(self.My)[:, None] * np.diag(self.Mx)[None, :] * F)

    def element_B(self, Ue, Ne, hx, hy):
        """Element contribution of int nu grad(phi).grad(u) by GLL quadrature:
        x part (h_y/h_x) D_x^T diag(nu w w) D_x u, y part likewise."""
        xi, w = gll(self.p)
        D = derivative_matrix(xi)
        ww = w[:, None] * w[None, :]
        Ux = Ue @ D.T          # d/dxi along columns (x)
        Uy = D @ Ue            # d/deta along rows (y)
        return ((hy / hx) * ww * Ne * Ux) @ D + D.T @ ((hx / hy) * ww * Ne * Uy)

    def element_nodes(self, ey, ex):
        p = self.p
        gy = [self.ay.node_index(ey, b) for b in range(p + 1)]
        gx = [self.ax.node_index(ex, a) for a in range(p + 1)]
        return gy, gx

    def apply_B(self, U, NU):
        """B(nu) u assembled from element quadrature of int nu grad(phi).grad(u)
        (Section 4, variable diffusion).  NU is the nodal diffusivity array."""
        U = self.zero_boundary(U)
        out = np.zeros(self.shape)
        for ey in range(self.ay.n):
            for ex in range(self.ax.n):
                gy, gx = self.element_nodes(ey, ex)
                Fe = self.element_B(U[np.ix_(gy, gx)], NU[np.ix_(gy, gx)],
                                    self.ax.h[ex], self.ay.h[ey])
                np.add.at(out, np.ix_(gy, gx), Fe)
        return self.zero_boundary(out)

    def dense_A(self):
        """Explicit A on the unknowns (row-major order), for small checks."""
        mx = self.ax.unknown_mask()
        my = self.ay.unknown_mask()
        Lx = self.Lx[np.ix_(mx, mx)]
        Mx = self.Mx[np.ix_(mx, mx)]
        Ly = self.Ly[np.ix_(my, my)]
        My = self.My[np.ix_(my, my)]
        return np.kron(My, Lx) + np.kron(Ly, Mx)

    def dense_B(self, NU):
        """Explicit B(nu) on the unknowns, assembled from element matrices
        (each obtained by applying the element operator to unit vectors)."""
        p = self.p
        num = -np.ones(self.shape, dtype=np.int64)
        num[self.mask] = np.arange(int(self.mask.sum()))
        n = int(self.mask.sum())
        B = np.zeros((n, n))
        for ey in range(self.ay.n):
            for ex in range(self.ax.n):
                gy, gx = self.element_nodes(ey, ex)
                Ne = NU[np.ix_(gy, gx)]
                ids = num[np.ix_(gy, gx)]
                for b in range(p + 1):
                    for a in range(p + 1):
                        if ids[b, a] < 0:
                            continue
                        E = np.zeros((p + 1, p + 1))
                        E[b, a] = 1.0
                        col = self.element_B(E, Ne, self.ax.h[ex], self.ay.h[ey])
                        for d in range(p + 1):
                            for c in range(p + 1):
                                if ids[d, c] >= 0:
                                    B[ids[d, c], ids[b, a]] += col[d, c]
        return B


def element_mean(space: Space, NU) -> np.ndarray:
    """nu_bar per element: the GLL-quadrature mean of nu over the element
    (Section 4: the local problems use the element average of nu).
    Returned as an (ny, nx) array."""
    p = space.p
    _, w = gll(p)
    out = np.zeros((space.ay.n, space.ax.n))
    for ey in range(space.ay.n):
        gy = [space.ay.node_index(ey, b) for b in range(p + 1)]
        for ex in range(space.ax.n):
            gx = [space.ax.node_index(ex, a) for a in range(p + 1)]
            out[ey, ex] = np.sum(w[:, None] * w[None, :] * NU[np.ix_(gy, gx)]) / 4.0
    return out
