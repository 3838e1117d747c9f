"""Extended-element subdomains and the weighted additive Schwarz smoother
(Section 3.1, Algorithm 2).

Subdomain of element e (per direction): the element's p+1 nodes plus n_o node
layers taken from each neighbour; the next node outward lies on the subdomain
boundary and is excluded, so in global node numbering the subdomain is
[e p - n_o, (e+1) p + n_o] (m = p + 1 + 2 n_o nodes).  With Dirichlet
boundaries, nodes on or beyond the domain boundary are not unknowns and are
dropped; with periodic boundaries indices wrap.

Local problem (eq. subproblem): A_ss du_s = r_s with A_ss = R_s A R_s^T, the
principal submatrix of A on the subdomain's unknowns.  Because the subdomain
is a Cartesian product of 1-D index sets, A_ss = M_sy (x) L_sx + L_sy (x) M_sx
with L_s*, M_s* the principal submatrices of the 1-D matrices.  The oracle
solves it with a dense factorisation (the definition); ``fdm_solve`` is the
paper's fast-diagonalisation formula, kept for the tests that pin the two
against each other.

Variable diffusion (Section 4): du_s ~ (1/nu_bar_s) A_ss^{-1} r_s with nu_bar_s
the mean of nu over the embedded element (eq. subproblem solution).

Combination (eq. correction global, Algorithm 2): u <- u + sum_s R_s^T W_s du_s
with W_s = W_y (x) W_x from the weight function, or W_s = R_s C^+ R_s^T with C
the counting matrix for arithmetic averaging.
"""
from __future__ import annotations

import numpy as np

from .discretization import DIRICHLET, PERIODIC, Axis, Space
from .weights import WF_ARITH, overlap_width, weight


class Subdomain1D:
    """Index set and extended coordinates of one subdomain in one direction."""

    def __init__(self, axis: Axis, L: np.ndarray, M: np.ndarray, e: int, n_o: int,
                 alpha_left: float = 1.0, alpha_right: float = 1.0):
        p = axis.p
        if not 0 <= n_o <= p - 1:
            raise ValueError("n_o must lie in [0, p-1]")
        xi = axis.xi
        self.e = e
        self.n_o = n_o
        self.m = p + 1 + 2 * n_o
        glob, xext, valid = [], [], []
        for t in range(-n_o, p + n_o + 1):
            if t < 0:
                x = xi[p + t] - 2.0          # node of the left neighbour
            elif t > p:
                x = xi[t - p] + 2.0          # node of the right neighbour
            else:
                x = xi[t]
            g = e * p + t
            if axis.bc == PERIODIC:
                g %= axis.N
                ok = True
            else:
                ok = 1 <= g <= axis.N - 2
            glob.append(g)
            xext.append(x)
            valid.append(ok)
        self.valid = np.array(valid)
        self.glob = np.array(glob)[self.valid]
        self.xi_ext = np.array(xext)[self.valid]
        self.Ls = L[np.ix_(self.glob, self.glob)]
        self.Ms = M[np.ix_(self.glob, self.glob)]
        delta = overlap_width(xi, n_o)
        self.delta_left = alpha_left * delta
        self.delta_right = alpha_right * delta
        self.left_sat = axis.bc == DIRICHLET and e == 0
        self.right_sat = axis.bc == DIRICHLET and e == axis.n - 1

    def key(self):
        return (self.Ls.shape[0], self.Ls.tobytes(), self.Ms.tobytes())

    def weights(self, kappa: int) -> np.ndarray:
        return weight(kappa, self.xi_ext, self.delta_left, self.delta_right,
                      self.left_sat, self.right_sat)


def local_matrix(sy: Subdomain1D, sx: Subdomain1D) -> np.ndarray:
    """A_ss = M_sy (x) L_sx + L_sy (x) M_sx (row-major: y slow, x fast)."""
    return np.kron(sy.Ms, sx.Ls) + np.kron(sy.Ls, sx.Ms)


def fdm_factors(Ls: np.ndarray, Ms: np.ndarray):
    """Generalised eigenproblem L_s S = M_s S Lambda with S^T M_s S = I
    (M_s is diagonal and positive)."""
    d = 1.0 / np.sqrt(np.diag(Ms))
    lam, Q = np.linalg.eigh(d[:, None] * Ls * d[None, :])
    return d[:, None] * Q, lam


def fdm_solve(sy: Subdomain1D, sx: Subdomain1D, Rs: np.ndarray) -> np.ndarray:
    """Fast diagonalisation (Section 3.1):
    A_ss^{-1} = (S_y (x) S_x)(I (x) Lambda_x + Lambda_y (x) I)^{-1}(S_y^T (x) S_x^T)."""
    Sx, lx = fdm_factors(sx.Ls, sx.Ms)
    Sy, ly = fdm_factors(sy.Ls, sy.Ms)
    T = Sy.T @ Rs @ Sx
    T = T / (ly[:, None] + lx[None, :])
    return Sy @ T @ Sx.T


class SchwarzLevel:
    """All subdomains of one level, grouped by identical local matrices."""

    def __init__(self, space: Space, n_o: int, wf: int = 5,
                 alpha_x=None, alpha_y=None):
        """alpha_x[I], alpha_y[J]: optional width scales per grid line
        (interface I between elements I-1 and I); 1 reproduces the paper."""
        self.space = space
        self.n_o = n_o
        self.wf = wf
        ax, ay = space.ax, space.ay
        nlx = ax.n + 1
        nly = ay.n + 1
        alpha_x = np.ones(nlx) if alpha_x is None else np.asarray(alpha_x, dtype=np.float64)
        alpha_y = np.ones(nly) if alpha_y is None else np.asarray(alpha_y, dtype=np.float64)
        if ax.bc == PERIODIC:
            alpha_x = alpha_x.copy()
            alpha_x[-1] = alpha_x[0]
        if ay.bc == PERIODIC:
            alpha_y = alpha_y.copy()
            alpha_y[-1] = alpha_y[0]
        self.sx = [Subdomain1D(ax, space.Lx, space.Mx, e, n_o, alpha_x[e], alpha_x[e + 1])
                   for e in range(ax.n)]
        self.sy = [Subdomain1D(ay, space.Ly, space.My, e, n_o, alpha_y[e], alpha_y[e + 1])
                   for e in range(ay.n)]
        if wf == WF_ARITH:
            self.count = counting_matrix(self)
        self._local_solvers()

    def _local_solvers(self):
        """Groups subdomains by their local matrices; one dense inverse per group."""
        ax, ay = self.space.ax, self.space.ay
        groups = {}
        for ey in range(ay.n):
            for ex in range(ax.n):
                k = (self.sy[ey].key(), self.sx[ex].key())
                groups.setdefault(k, []).append((ey, ex))
        self.groups = []
        for members in groups.values():
            ey0, ex0 = members[0]
            A_ss = local_matrix(self.sy[ey0], self.sx[ex0])
            Ainv = np.linalg.inv(A_ss)
            gy = np.array([self.sy[ey].glob for ey, _ in members])
            gx = np.array([self.sx[ex].glob for _, ex in members])
            W = np.array([self.subdomain_weights(ey, ex) for ey, ex in members])
            self.groups.append((members, Ainv, gy, gx, W))

    def subdomain_weights(self, ey: int, ex: int) -> np.ndarray:
        sy, sx = self.sy[ey], self.sx[ex]
        if self.wf == WF_ARITH:
            return 1.0 / self.count[np.ix_(sy.glob, sx.glob)]
        return np.outer(sy.weights(self.wf), sx.weights(self.wf))

    def corrections(self, R: np.ndarray, nubar=None) -> np.ndarray:
        """sum_s R_s^T W_s A_ss^{-1} R_s r (divided by nu_bar_s if given)."""
        dU = np.zeros(self.space.shape)
        for members, Ainv, gy, gx, W in self.groups:
            Rs = R[gy[:, :, None], gx[:, None, :]]
            n, my, mx = Rs.shape
            D = (Rs.reshape(n, my * mx) @ Ainv.T).reshape(n, my, mx)
            if nubar is not None:
                D = D / np.array([nubar[ey, ex] for ey, ex in members])[:, None, None]
            np.add.at(dU, (gy[:, :, None], gx[:, None, :]), W * D)
        return dU

    def smooth(self, U, F, n_it: int, NU=None, nubar=None):
        """Algorithm 2 (WSchwarz): n_it sweeps of r = f - A u, u += sum_s ...
        With NU given, the residual uses B(nu) and the local solves nu_bar."""
        sp = self.space
        for _ in range(n_it):
            R = F - (sp.apply_A(U) if NU is None else sp.apply_B(U, NU))
            R = sp.zero_boundary(R)
            U = U + self.corrections(R, nubar)
        return U


def counting_matrix(level: SchwarzLevel) -> np.ndarray:
    """C = sum_s R_s^T R_s: how many subdomains contain each unknown."""
    C = np.zeros(level.space.shape)
    for sy in level.sy:
        for sx in level.sx:
            C[np.ix_(sy.glob, sx.glob)] += 1.0
    C[~level.space.mask] = 1.0
    return C


class ElementwiseSchwarzLevel:
    """Weighted additive Schwarz with parameters chosen per element (the
    learned-parameter extension; the paper fixes one overlap per level and one
    weight width).  Element e has its own overlap n_o,e and width scale
    alpha_e: its subdomain is the window of Section 3.1 with n_o,e layers, and
    its 1-D weights are the weight function with delta = alpha_e delta_o(n_o,e)
    on both sides (saturated at Dirichlet sides).  Neighbouring subdomains then
    no longer share their transition zones, so the weights need not sum to
    one; the correction is normalised node by node (Shepard):

        u <- u + D^{-1} sum_s R_s^T W_s du_s,   D = sum_s R_s^T W_s R_s,

    which is a partition of unity by construction and reduces to the paper's
    update when every element carries the same parameters (then D = 1).
    With unit weights (the arithmetic mean of Table 1) D is the counting
    matrix C and D^{-1} W_s = R_s C^+ R_s^T."""

    def __init__(self, space: Space, elem_no, elem_alpha, wf: int = 5):
        self.space = space
        self.wf = wf
        ax, ay = space.ax, space.ay
        elem_no = np.asarray(elem_no, dtype=int)
        elem_alpha = np.asarray(elem_alpha, dtype=np.float64)
        assert elem_no.shape == (ay.n, ax.n) and elem_alpha.shape == (ay.n, ax.n)
        self.elem_no = elem_no
        self.elem_alpha = elem_alpha
        self.sub = {}
        D = np.zeros(space.shape)
        for ey in range(ay.n):
            for ex in range(ax.n):
                n_o, a = int(elem_no[ey, ex]), float(elem_alpha[ey, ex])
                sx = Subdomain1D(ax, space.Lx, space.Mx, ex, n_o, a, a)
                sy = Subdomain1D(ay, space.Ly, space.My, ey, n_o, a, a)
                if wf == WF_ARITH:
                    W = np.ones((len(sy.glob), len(sx.glob)))
                else:
                    W = np.outer(sy.weights(wf), sx.weights(wf))
                Ainv = np.linalg.inv(local_matrix(sy, sx))
                self.sub[ey, ex] = (sy, sx, W, Ainv)
                D[np.ix_(sy.glob, sx.glob)] += W
        D[~space.mask] = 1.0
        self.D = D

    def corrections(self, R: np.ndarray, nubar=None) -> np.ndarray:
        """D^{-1} sum_s R_s^T W_s A_ss^{-1} R_s r (divided by nu_bar_s if given)."""
        dU = np.zeros(self.space.shape)
        for (ey, ex), (sy, sx, W, Ainv) in self.sub.items():
            Rs = R[np.ix_(sy.glob, sx.glob)]
            d = (Ainv @ Rs.ravel()).reshape(Rs.shape)
            if nubar is not None:
                d = d / nubar[ey, ex]
            dU[np.ix_(sy.glob, sx.glob)] += W * d
        return dU / self.D

    def smooth(self, U, F, n_it: int, NU=None, nubar=None):
        sp = self.space
        for _ in range(n_it):
            R = F - (sp.apply_A(U) if NU is None else sp.apply_B(U, NU))
            R = sp.zero_boundary(R)
            U = U + self.corrections(R, nubar)
        return U


class MultiplicativeSchwarzLevel:
    """Multiplicative Schwarz method (Section 3.1, Algorithm 1): the subdomain
    problems are solved one after the other, each on the residual left by all
    the corrections before it, without weights.  Sweep i visits the elements
    in order e = 1 .. n_el when i is odd and in reverse when i is even, so an
    even number of sweeps is a symmetric smoother.  Reading: the elements are
    numbered row by row, e = ey nx + ex (x fastest).  Variable diffusion uses
    B(nu) in the residual and nu_bar_s in the local solve, as the additive
    method does."""

    def __init__(self, space: Space, n_o: int):
        self.space = space
        self.n_o = n_o
        ax, ay = space.ax, space.ay
        self.sx = [Subdomain1D(ax, space.Lx, space.Mx, e, n_o) for e in range(ax.n)]
        self.sy = [Subdomain1D(ay, space.Ly, space.My, e, n_o) for e in range(ay.n)]
        self.inv = {}
        for ey in range(ay.n):
            for ex in range(ax.n):
                k = (self.sy[ey].key(), self.sx[ex].key())
                if k not in self.inv:
                    self.inv[k] = np.linalg.inv(local_matrix(self.sy[ey], self.sx[ex]))
        self.order = [(ey, ex) for ey in range(ay.n) for ex in range(ax.n)]

    def smooth(self, U, F, n_it: int, NU=None, nubar=None):
        sp = self.space
        U = np.array(U, dtype=np.float64)
        for i in range(1, n_it + 1):
            seq = self.order if i % 2 == 1 else self.order[::-1]
            for ey, ex in seq:
                R = F - (sp.apply_A(U) if NU is None else sp.apply_B(U, NU))
                sy, sx = self.sy[ey], self.sx[ex]
                Rs = R[np.ix_(sy.glob, sx.glob)]
                d = (self.inv[(sy.key(), sx.key())] @ Rs.ravel()).reshape(Rs.shape)
                if nubar is not None:
                    d = d / nubar[ey, ex]
                U[np.ix_(sy.glob, sx.glob)] += d
            U = sp.zero_boundary(U)
        return U


def window_nodes(axis: Axis, e: int, n_o: int):
    """Positions t of the window [e p - n_o, (e+1) p + n_o] of subdomain e that
    are mesh nodes (with Dirichlet ends, positions beyond the boundary node
    are not), and their global node indices.  The positions form a range."""
    p = axis.p
    pos, glob = [], []
    for t in range(p + 1 + 2 * n_o):
        g = e * p - n_o + t
        if axis.bc == PERIODIC:
            g %= axis.N
        elif not 0 <= g <= axis.N - 1:
            continue
        pos.append(t)
        glob.append(g)
    return pos, glob


def weighted_axis_matrices(axis: Axis, e: int, n_o: int, coef) -> tuple:
    """1-D stiffness and lumped mass around subdomain e with a coefficient
    given per window position, assembled over the elements e - 1, e, e + 1
    (clipped at Dirichlet ends, wrapped when periodic) by GLL quadrature:
        L^E_ab = (2/h) sum_q w_q c_q D_qa D_qb,   M^E_aa = (h/2) w_a c_a,
    where local node q of element e + d sits at window position d p + q + n_o
    and c_q = coef(that position clamped to the window's node range).
    Dense N x N over all global nodes."""
    from .gll import derivative_matrix
    p = axis.p
    w = axis.w
    D = derivative_matrix(axis.xi)
    pos, _ = window_nodes(axis, e, n_o)
    L = np.zeros((axis.N, axis.N))
    M = np.zeros((axis.N, axis.N))
    for d in (-1, 0, 1):
        E = e + d
        if axis.bc == PERIODIC:
            E %= axis.n
        elif not 0 <= E < axis.n:
            continue
        idx = [axis.node_index(E, q) for q in range(p + 1)]
        c = np.array([coef(min(max(d * p + q + n_o, pos[0]), pos[-1])) for q in range(p + 1)])
        Le = (2.0 / axis.h[E]) * (D.T @ ((w * c)[:, None] * D))
        for qa in range(p + 1):
            M[idx[qa], idx[qa]] += 0.5 * axis.h[E] * w[qa] * c[qa]
            for qb in range(p + 1):
                L[idx[qa], idx[qb]] += Le[qa, qb]
    return L, M


def separable_fit(LG: np.ndarray):
    """Least-squares split of a grid function into a function of the column
    plus a function of the row, LG[j, i] ~ alpha_i + beta_j, with every grid
    point weighted equally: alpha_i = (column mean)_i - (grand mean),
    beta_j = (row mean)_j."""
    g = LG.mean()
    return LG.mean(axis=0) - g, LG.mean(axis=1)


class SeparableSchwarzLevel(SchwarzLevel):
    """Weighted additive Schwarz for variable diffusion with separable local
    coefficients (a project extension; Section 4 replaces nu by its element
    mean in the local problems, which fails where nu varies strongly inside a
    subdomain).  For subdomain s, log nu on the window's nodes is fitted by
    least squares as alpha(x) + beta(y) (separable_fit), and the local
    operator is the restriction of B(nu_s) with nu_s = a(x) b(y),
    a = exp(alpha), b = exp(beta), extended beyond the window (into the parts
    of the neighbouring elements that the window does not cover) by the value
    at the window's nearest node.  That operator is exactly separable,

        A_s = R_s [M_b (x) L_a + L_b (x) M_a] R_s^T,

    with L_a, M_a the 1-D stiffness and mass weighted by a (GLL quadrature;
    weighted_axis_matrices), so the fast diagonalisation still applies, with
    factors per subdomain.  Subdomains, weights and the update are the
    paper's (Algorithm 2); there is no 1/nu_bar scaling.  Periodic
    directions need at least 3 elements (the window then meets each
    neighbouring element at one end only)."""

    def __init__(self, space: Space, n_o: int, wf: int, NU):
        self.NU = np.asarray(NU, dtype=np.float64)
        for ax_ in (space.ax, space.ay):
            if ax_.bc == PERIODIC and ax_.n < 3:
                raise ValueError("separable local solves need 3 elements per periodic direction")
        super().__init__(space, n_o, wf)

    def coefficients(self, ey: int, ex: int):
        """(a, b): dicts from window position to the fitted factors."""
        ax, ay = self.space.ax, self.space.ay
        px, gx = window_nodes(ax, ex, self.n_o)
        py, gy = window_nodes(ay, ey, self.n_o)
        alpha, beta = separable_fit(np.log(self.NU[np.ix_(gy, gx)]))
        return dict(zip(px, np.exp(alpha))), dict(zip(py, np.exp(beta)))

    def local_matrix_of(self, ey: int, ex: int) -> np.ndarray:
        ax, ay = self.space.ax, self.space.ay
        a, b = self.coefficients(ey, ex)
        La, Ma = weighted_axis_matrices(ax, ex, self.n_o, a.__getitem__)
        Lb, Mb = weighted_axis_matrices(ay, ey, self.n_o, b.__getitem__)
        ix, iy = self.sx[ex].glob, self.sy[ey].glob
        return (np.kron(Mb[np.ix_(iy, iy)], La[np.ix_(ix, ix)])
                + np.kron(Lb[np.ix_(iy, iy)], Ma[np.ix_(ix, ix)]))

    def _local_solvers(self):
        self.inv = {}
        for ey in range(self.space.ay.n):
            for ex in range(self.space.ax.n):
                self.inv[ey, ex] = np.linalg.inv(self.local_matrix_of(ey, ex))

    def corrections(self, R: np.ndarray, nubar=None) -> np.ndarray:
        """sum_s R_s^T W_s A_s^{-1} R_s r (nubar is not used: the coefficient
        is inside A_s)."""
        dU = np.zeros(self.space.shape)
        for (ey, ex), Ainv in self.inv.items():
            sy, sx = self.sy[ey], self.sx[ex]
            Rs = R[np.ix_(sy.glob, sx.glob)]
            d = (Ainv @ Rs.ravel()).reshape(Rs.shape)
            dU[np.ix_(sy.glob, sx.glob)] += self.subdomain_weights(ey, ex) * d
        return dU
