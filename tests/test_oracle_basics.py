"""Pins of the oracle's discretisation against closed forms and invariants
(Section 2; GLL quadrature, Lagrange derivative, SEM operators)."""
import math

import numpy as np
import pytest

from oracle.discretization import DIRICHLET, PERIODIC, Axis, Space, element_mean
from oracle.gll import derivative_matrix, element_matrices, gll, lagrange_matrix
from paper_1512_02390_amd import workloads as W


def test_gll_closed_forms():
    x, w = gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = gll(4)
    s = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", list(range(1, 33)))
def test_gll_exactness(p):
    """GLL with p+1 points integrates x^k exactly for k <= 2p-1, not x^(2p)."""
    x, w = gll(p)
    assert np.allclose(x, -x[::-1], atol=1e-14) and np.allclose(w, w[::-1], atol=1e-14)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 2e-14 * max(1, p / 4)
    if p <= 10:
        k = 2 * p
        assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 16])
def test_derivative_exact_on_polynomials(p):
    x, _ = gll(p)
    D = derivative_matrix(x)
    for k in range(p + 1):
        d = k * x ** (k - 1) if k else np.zeros_like(x)
        assert np.allclose(D @ x ** k, d, atol=1e-11 * (1 + p))


def test_element_matrices_closed_forms():
    L1, _, _, _, _ = element_matrices(1)
    assert np.allclose(L1, 0.5 * np.array([[1, -1], [-1, 1]]), atol=1e-15)
    L2, _, _, _, _ = element_matrices(2)
    assert np.allclose(L2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 6, atol=1e-14)
    for p in (3, 7, 12):
        L, _, _, _, _ = element_matrices(p)
        assert np.allclose(L.sum(axis=1), 0, atol=1e-12)
        assert np.allclose(L, L.T, atol=1e-13)


def test_lagrange_matrix_interpolates():
    x, _ = gll(6)
    t = np.linspace(-1, 1, 13)
    E = lagrange_matrix(x, t)
    for k in range(7):
        assert np.allclose(E @ x ** k, t ** k, atol=1e-13)


def test_p1_eigenvalues_closed_form():
    """p = 1, lumped mass, Dirichlet: generalised eigenvalues (4/h^2) sin^2(k pi / 2n)."""
    n, length = 9, 1.7
    ax = Axis(W.uniform_breaks(n, length), 1, DIRICHLET)
    L, M = ax.assemble()
    Li, Mi = L[1:-1, 1:-1], M[1:-1, 1:-1]
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(Mi, Li)).real)
    h = length / n
    ref = (4 / h ** 2) * np.sin(np.arange(1, n) * math.pi / (2 * n)) ** 2
    assert np.allclose(lam, ref, rtol=1e-12)


@pytest.mark.parametrize("bc", [DIRICHLET, PERIODIC])
def test_kronecker_equals_element_quadrature(bc):
    """A = M_y (x) L_x + L_y (x) M_x equals the element-by-element GLL Galerkin
    matrix B(1) on a stretched mesh."""
    xb = W.geometric_breaks(3, 0.3, 4.0)
    yb = np.array([0.0, 0.2, 0.7, 1.0])
    sp = Space(xb, yb, 3, bc)
    A = sp.dense_A()
    B = sp.dense_B(np.ones(sp.shape))
    assert np.allclose(A, B, atol=1e-12 * np.abs(A).max())
    U = W.random_guess(sp.shape, bc, 5)
    assert np.allclose(sp.apply_A(U), sp.apply_B(U, np.ones(sp.shape)), atol=1e-12)


def test_operator_symmetry_definiteness_nullspace():
    xb = W.uniform_breaks(3, 1.0)
    sd = Space(xb, xb, 4, DIRICHLET)
    A = sd.dense_A()
    assert np.allclose(A, A.T, atol=1e-13)
    assert np.linalg.eigvalsh(A).min() > 0
    sp = Space(xb, xb, 4, PERIODIC)
    A = sp.dense_A()
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-10 and ev[1] > 1e-3
    assert np.allclose(A @ np.ones(A.shape[0]), 0, atol=1e-12)


def test_variable_nu_operator():
    """B(c) = c A; B(nu) symmetric, with the constants in its null space
    when periodic."""
    xb = W.uniform_breaks(3, 1.0)
    sp = Space(xb, xb, 3, PERIODIC)
    U = W.random_guess(sp.shape, PERIODIC, 4)
    assert np.allclose(sp.apply_B(U, 2.5 * np.ones(sp.shape)), 2.5 * sp.apply_A(U), atol=1e-12)
    nu = W.PaperNu(0.9)
    NU = W.nodal(nu.nu, sp.x(), sp.y())
    B = sp.dense_B(NU)
    assert np.allclose(B, B.T, atol=1e-12)
    assert np.allclose(B @ np.ones(B.shape[0]), 0, atol=1e-11)
    nb = element_mean(sp, NU)
    assert nb.shape == (3, 3) and np.all(nb > 0.1)
    # element mean of a function that is constant per element reproduces it
    assert np.allclose(element_mean(sp, 3.0 * np.ones(sp.shape)), 3.0)


@pytest.mark.parametrize("p", [3, 4, 7])
def test_element_mean_of_polynomial_field_is_exact(p):
    """nu_bar_e (Section 4) is the mean of nu over the element.  For a field
    that is a polynomial of degree <= 2p - 1 in each variable the GLL rule is
    exact, so on a stretched mesh nu_bar_e equals the closed-form mean
    (1 / |e|) int_e nu.  A plain average of the nodal values fails this."""
    xb = W.geometric_breaks(4, 0.2, 3.0)
    yb = np.array([0.0, 0.15, 0.5, 1.3])
    sp = Space(xb, yb, p, DIRICHLET)

    def nu(x, y):
        return 1.0 + x ** 2 * y + 3.0 * y ** 3 + 0.5 * x ** 5 * y ** 2

    def mean_pow(a, b, k):
        return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))

    NU = W.nodal(nu, sp.x(), sp.y())
    got = element_mean(sp, NU)
    for ey in range(len(yb) - 1):
        for ex in range(len(xb) - 1):
            a, b, c, d = xb[ex], xb[ex + 1], yb[ey], yb[ey + 1]
            exact = (1.0 + mean_pow(a, b, 2) * mean_pow(c, d, 1) + 3.0 * mean_pow(c, d, 3)
                     + 0.5 * mean_pow(a, b, 5) * mean_pow(c, d, 2))
            assert abs(got[ey, ex] - exact) < 1e-13 * exact
    # the unweighted nodal average is a different number on these elements
    gy = [sp.ay.node_index(1, b) for b in range(p + 1)]
    gx = [sp.ax.node_index(2, a) for a in range(p + 1)]
    assert abs(NU[np.ix_(gy, gx)].mean() - got[1, 2]) > 1e-3 * got[1, 2]


def _solve_dirichlet(n, p):
    xb = W.uniform_breaks(n, 1.0)
    sp = Space(xb, xb, p, DIRICHLET)
    sol = W.SineSolution()
    F = sp.mass(-W.nodal(sol.laplacian, sp.x(), sp.y()))
    A = sp.dense_A()
    u = np.linalg.solve(A, F[sp.mask])
    ue = W.nodal(sol.u, sp.x(), sp.y())[sp.mask]
    return np.abs(u - ue).max()


def test_spectral_convergence_in_p():
    """Manufactured u = sin(pi x) sin(pi y) on 4x4 elements: the nodal error
    falls exponentially with p (until rounding)."""
    errs = [_solve_dirichlet(4, p) for p in (2, 3, 4, 5, 6, 7)]
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < a / 5
    assert errs[-1] < 1e-8
    assert _solve_dirichlet(4, 10) < 1e-12


def test_algebraic_convergence_in_h():
    for p in (2, 3):
        e1, e2 = _solve_dirichlet(4, p), _solve_dirichlet(8, p)
        assert math.log2(e1 / e2) > p + 1 - 0.5


def _solve_varnu(p):
    """-div(nu grad u) = f on [0,1]^2 (Dirichlet) with u = sin(pi x) sin(pi y)
    and nu = 1 + x/2 + y^2/4 (not symmetric in x and y), on 3x3 elements of
    unequal widths in x; f worked out by hand:
      f = -(nu_x u_x + nu_y u_y) + 2 pi^2 nu u,  nu_x = 1/2, nu_y = y/2."""
    pi = math.pi
    xb = np.array([0.0, 0.2, 0.55, 1.0])
    yb = W.uniform_breaks(3, 1.0)
    sp = Space(xb, yb, p, DIRICHLET)
    nu = lambda x, y: 1.0 + 0.5 * x + 0.25 * y * y
    u = lambda x, y: np.sin(pi * x) * np.sin(pi * y)
    ux = lambda x, y: pi * np.cos(pi * x) * np.sin(pi * y)
    uy = lambda x, y: pi * np.sin(pi * x) * np.cos(pi * y)
    f = lambda x, y: -(0.5 * ux(x, y) + 0.5 * y * uy(x, y)) + 2 * pi * pi * nu(x, y) * u(x, y)
    NU = W.nodal(nu, sp.x(), sp.y())
    F = sp.mass(W.nodal(f, sp.x(), sp.y()))
    U = np.linalg.solve(sp.dense_B(NU), F[sp.mask])
    return np.abs(U - W.nodal(u, sp.x(), sp.y())[sp.mask]).max()


def test_variable_nu_spectral_convergence():
    """B(nu) against a manufactured solution with an asymmetric nu on
    stretched elements: exponential convergence in p to near rounding, so a
    transposed nu, a wrong Jacobian factor or a wrong quadrature weight in
    the variable-coefficient term cannot pass."""
    errs = [_solve_varnu(p) for p in (3, 5, 7, 9)]
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < a / 20
    assert errs[-1] < 1e-7
