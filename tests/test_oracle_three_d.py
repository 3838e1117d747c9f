"""Pins of the 3-D oracle (the conclusions' 3-D extension): the operator by
two routes and by a manufactured solution, the Schwarz partition of unity and
exact single-element solve, the 3-D fast diagonalisation, the transfers, and
MGCG against textbook CG."""
import numpy as np
import pytest

from oracle.mgcg import mgcg
from oracle.three_d import Multigrid3, SchwarzLevel3, Space3, fdm_solve3, local_matrix3
from paper_1512_02390_amd import workloads as W


def _mesh(stretched=True):
    if stretched:
        return W.geometric_breaks(3, 0.3, 2.0), W.uniform_breaks(2, 1.0), W.geometric_breaks(2, 0.4, 1.5)
    return W.uniform_breaks(2, 1.0), W.uniform_breaks(2, 1.0), W.uniform_breaks(2, 1.0)


def test_operator_axes_match_kronecker_form():
    xb, yb, zb = _mesh()
    sp = Space3(xb, yb, zb, 3)
    rng = np.random.default_rng(0)
    U = sp.zero_boundary(rng.normal(size=sp.shape))
    A = sp.dense_A()
    assert np.allclose(sp.apply_A(U)[sp.mask], A @ U[sp.mask], rtol=0, atol=1e-12 * np.abs(A).max())
    # symmetric positive definite
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0


def test_manufactured_solution_converges_spectrally():
    """-lap u = 3 pi^2 u for u = sin(pi x) sin(pi y) sin(pi z) on the unit cube:
    the discrete solution's nodal error falls by orders of magnitude from p = 3
    to p = 7 (a wrong mass or stiffness scale along any axis stalls it)."""
    errs = []
    for p in (3, 5, 7):
        sp = Space3(W.uniform_breaks(2, 1.0), W.geometric_breaks(2, 0.4, 1.5), W.uniform_breaks(2, 1.0), p)
        x, y, z = sp.coords()
        uex = (np.sin(np.pi * z)[:, None, None] * np.sin(np.pi * y)[None, :, None]
               * np.sin(np.pi * x)[None, None, :])
        b = sp.mass(3 * np.pi ** 2 * uex)
        A = sp.dense_A()
        u = np.linalg.solve(A, b[sp.mask])
        errs.append(np.abs(u - uex[sp.mask]).max())
    assert errs[0] > 30 * errs[1] > 30 * 30 * errs[2], errs
    assert errs[2] < 1e-5


@pytest.mark.parametrize("p,n_o,wf", [(3, 1, 5), (4, 2, 3), (6, 1, 1), (5, 0, 7), (4, 3, -1)])
def test_partition_of_unity(p, n_o, wf):
    xb, yb, zb = _mesh()
    lev = SchwarzLevel3(Space3(xb, yb, zb, p), n_o, wf)
    S = np.zeros(lev.space.shape)
    for ez, sz in enumerate(lev.sz):
        for ey, sy in enumerate(lev.sy):
            for ex, sx in enumerate(lev.sx):
                S[np.ix_(sz.glob, sy.glob, sx.glob)] += lev.weights(ez, ey, ex)
    assert np.allclose(S[lev.space.mask], 1.0, atol=1e-14)


def test_single_element_smoother_is_exact_solve():
    sp = Space3([0.0, 1.3], [0.0, 0.7], [0.0, 1.0], 5)
    lev = SchwarzLevel3(sp, 2, 5)
    rng = np.random.default_rng(1)
    F = sp.zero_boundary(rng.normal(size=sp.shape))
    U = lev.smooth(np.zeros(sp.shape), F, 1)
    assert np.abs(sp.apply_A(U) - F)[sp.mask].max() <= 1e-11 * np.abs(F).max()


def test_fast_diagonalisation_equals_dense_local_inverse():
    xb, yb, zb = _mesh()
    lev = SchwarzLevel3(Space3(xb, yb, zb, 4), 1, 5)
    rng = np.random.default_rng(2)
    for ez, ey, ex in [(0, 0, 0), (1, 1, 2), (0, 1, 1)]:
        sz, sy, sx = lev.sz[ez], lev.sy[ey], lev.sx[ex]
        Rs = rng.normal(size=(len(sz.glob), len(sy.glob), len(sx.glob)))
        ref = (np.linalg.inv(local_matrix3(sz, sy, sx)) @ Rs.ravel()).reshape(Rs.shape)
        assert np.allclose(fdm_solve3(sz, sy, sx, Rs), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_transfers_reproduce_coarse_polynomials_and_are_adjoint():
    xb, yb, zb = _mesh()
    mg = Multigrid3(xb, yb, zb, 6, 0, 1)
    for l in range(1, mg.L + 1):
        sc, sf = mg.spaces[l - 1], mg.spaces[l]
        q = sc.p
        xc, yc, zc = sc.coords()
        xf, yf, zf = sf.coords()
        Uc = (zc ** min(q, 1))[:, None, None] * (yc ** min(q, 2))[None, :, None] * (xc ** q)[None, None, :]
        Uf = (zf ** min(q, 1))[:, None, None] * (yf ** min(q, 2))[None, :, None] * (xf ** q)[None, None, :]
        Px, Py, Pz = mg.P[l]
        from oracle.three_d import _along
        assert np.allclose(_along(Pz, _along(Py, _along(Px, Uc, 2), 1), 0), Uf, atol=1e-11)
        rng = np.random.default_rng(l)
        R = sf.zero_boundary(rng.normal(size=sf.shape))
        V = sc.zero_boundary(rng.normal(size=sc.shape))
        assert abs(np.vdot(mg.restrict(l, R), V) - np.vdot(R, mg.prolong(l, V))) < 1e-11 * np.abs(R).sum()


def test_mgcg_without_preconditioner_is_textbook_cg():
    from oracle.mgcg import textbook_pcg
    xb, yb, zb = _mesh()
    mg = Multigrid3(xb, yb, zb, 3, 0, 1)
    sp = mg.spaces[-1]
    rng = np.random.default_rng(3)
    F = sp.zero_boundary(rng.normal(size=sp.shape))
    U0 = sp.zero_boundary(rng.uniform(size=sp.shape))
    U, hist, it = mgcg(mg, U0, F, 12, 1e-30, precond=lambda r: r.copy())
    xs = textbook_pcg(sp.dense_A(), F[sp.mask], U0[sp.mask], lambda r: r.copy(), 12, 1e-30)
    assert np.allclose(U[sp.mask], xs[-1], rtol=0, atol=1e-10 * np.abs(xs[-1]).max())


def test_mgcg_converges_with_schwarz_multigrid():
    xb, yb, zb = _mesh()
    mg = Multigrid3(xb, yb, zb, 8, 1, 0)     # ceil(p_l / 8) overlaps
    sp = mg.spaces[-1]
    F = sp.mass(sp.zero_boundary(np.random.default_rng(5).uniform(-1, 1, size=sp.shape)))
    U0 = sp.zero_boundary(np.random.default_rng(6).uniform(size=sp.shape))
    U, hist, it = mgcg(mg, U0, F, 40, 1e-10)
    assert hist[-1] <= 1e-10 * hist[0] and it <= 20, (it, hist[-1] / hist[0])
    # the recursion's residual is the true one
    assert np.linalg.norm(mg.residual(mg.L, U, F)[sp.mask]) <= 1.5e-10 * hist[0]
