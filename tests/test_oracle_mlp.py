"""Pins of the learned-parameter oracle (oracle/mlp.py): gradients against
central differences, closed forms of the network and of Adam's first step,
closed forms and symmetries of the element features, hand-computed reductions
of predictions to solver parameters, and the cost measure against the paper's
omega formula (itself pinned against Tables 4 and 5)."""
import math

import numpy as np
import pytest

from oracle import mlp
from oracle.metrics import omega_k
from oracle.multigrid import level_orders
from paper_1512_02390_amd import workloads as W


def _data(n=7, seed=5):
    g = W.rng(seed)
    return g.normal(size=(n, mlp.D_IN)), g.uniform(0.05, 0.95, size=(n, mlp.D_OUT))


def test_param_count_and_packing():
    th = W.mlp_init()
    assert th.size == mlp.n_params() == 64 * 8 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    assert W1.shape == (64, 8) and W3.shape == (2, 64)
    assert not b1.any() and not b2.any() and not b3.any()


def test_gradient_matches_central_differences():
    th = W.mlp_init() + 0.05 * W.rng(9).normal(size=mlp.n_params())
    X, T = _data()
    L, g = mlp.gradient(th, X, T)
    assert L == pytest.approx(mlp.loss(th, X, T), rel=1e-14)
    h = 1e-6
    fd = np.zeros_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd[i] = (mlp.loss(th + e, X, T) - mlp.loss(th - e, X, T)) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)
    # each block of parameters is exercised
    for part in mlp.unpack(g):
        assert np.abs(part).max() > 0


def test_zero_weights_closed_form():
    th = np.zeros(mlp.n_params())
    b3 = np.array([0.3, -1.2])
    th[-2:] = b3
    X, T = _data()
    Y, _ = mlp.forward(th, X)
    s = 1.0 / (1.0 + np.exp(-b3))
    assert np.allclose(Y, s[None, :], rtol=0, atol=1e-15)
    _, g = mlp.gradient(th, X, T)
    gb3 = ((s[None, :] - T) * s * (1 - s)).sum(0) / len(X)
    assert np.allclose(g[-2:], gb3, rtol=1e-14)
    assert not g[:-2].any()       # every other gradient carries a zero factor


def test_adam_first_step_is_normalised_gradient():
    th = W.mlp_init()
    X, T = _data()
    _, g = mlp.gradient(th, X, T)
    opt = mlp.Adam(th)
    new = opt.step(g, 1e-3)
    assert np.allclose(th - new, 1e-3 * g / (np.abs(g) + mlp.EPS), rtol=1e-12, atol=0)


def test_training_reduces_loss():
    g = W.rng(11)
    X = g.normal(size=(64, mlp.D_IN))
    T = np.stack([1 / (1 + np.exp(-X[:, 0])), 0.5 + 0.4 * np.tanh(X[:, 1] * X[:, 2])], 1)
    opt = mlp.Adam(W.mlp_init())
    L0, _ = mlp.gradient(opt.theta, X, T)
    for _ in range(300):
        _, gr = mlp.gradient(opt.theta, X, T)
        opt.step(gr, 3e-3)
    L1, _ = mlp.gradient(opt.theta, X, T)
    assert L1 < 0.1 * L0


def test_features_uniform_constant_nu():
    xb, yb = W.uniform_breaks(3, 1.5), W.uniform_breaks(2, 1.0)
    F = mlp.element_features(xb, yb, 4, W.BC_DIRICHLET, None)
    assert F.shape == (6, 8)
    assert np.allclose(F[:, 0], math.log2(0.5 / 0.5))
    assert np.allclose(F[:, 1:7], 0.0, atol=1e-14)
    assert np.allclose(F[:, 7], 4 / 32)
    # a constant nu = c moves only feature 1
    from oracle.discretization import Space
    c = 3.7
    Fc = mlp.element_features(xb, yb, 4, W.BC_DIRICHLET, np.full(Space(xb, yb, 4, 0).shape, c))
    assert np.allclose(Fc[:, 1], math.log(c), atol=1e-14)
    assert np.allclose(np.delete(Fc, 1, axis=1), np.delete(F, 1, axis=1), atol=1e-14)


def test_features_aspect_ratio_and_exponential_nu():
    from oracle.discretization import Space
    xb = W.geometric_breaks(4, 0.25, 8.0)
    yb = W.uniform_breaks(3, 1.0)
    p = 5
    sp = Space(xb, yb, p, W.BC_DIRICHLET)
    a, b = 0.7, -1.3
    NU = np.exp(a * sp.x()[None, :] + b * sp.y()[:, None])
    F = mlp.element_features(xb, yb, p, W.BC_DIRICHLET, NU)
    hx, hy = np.diff(xb), np.diff(yb)
    for ey in range(3):
        for ex in range(4):
            e = ey * 4 + ex
            assert F[e, 0] == pytest.approx(math.log2(hx[ex] / hy[ey]), abs=1e-14)
            # nu is monotone in x and y: max / min at opposite corners
            assert F[e, 6] == pytest.approx(a * hx[ex] + abs(b) * hy[ey], rel=1e-12)
    # neighbour contrasts are antisymmetric and vanish at Dirichlet sides
    G = F.reshape(3, 4, 8)
    assert np.allclose(G[:, :-1, 3], -G[:, 1:, 2], atol=1e-14)
    assert np.allclose(G[:-1, :, 5], -G[1:, :, 4], atol=1e-14)
    assert not G[:, 0, 2].any() and not G[:, -1, 3].any()
    assert not G[0, :, 4].any() and not G[-1, :, 5].any()


def test_features_periodic_wrap():
    from oracle.discretization import Space
    xb, yb = W.uniform_breaks(3, 1.0), W.uniform_breaks(3, 1.0)
    sp = Space(xb, yb, 3, W.BC_PERIODIC)
    NU = np.exp(np.sin(2 * math.pi * sp.x())[None, :] + 0 * sp.y()[:, None])
    G = mlp.element_features(xb, yb, 3, W.BC_PERIODIC, NU).reshape(3, 3, 8)
    assert np.allclose(G[:, 0, 2], -G[:, -1, 3], atol=1e-14)
    assert np.allclose(G[:, :, 4:6], 0.0, atol=1e-14)   # nu constant along y


def test_setup_from_predictions_hand_example():
    pred = np.array([[0.5, 0.5], [1.0, 1.0]])          # nx = 2, ny = 1
    ov, ax, ay = mlp.setup_from_predictions(pred, 2, 1, 8, W.BC_DIRICHLET)
    # rho = 0.5 * 0.75 = 0.375; levels p = 1, 2, 4, 8
    assert ov == [0, 1, 2, 3]
    assert np.allclose(ax, [0.5, 0.75, 1.0])
    assert np.allclose(ay, [0.75, 0.75])
    # alpha clipped to [0.1, 1]; overlap capped by the 48-node tile at p = 32
    ov, ax, ay = mlp.setup_from_predictions([[0.01, 1.0]], 1, 1, 32, W.BC_DIRICHLET)
    assert ov == [0, 1, 2, 4, 8, 7]
    assert np.allclose(ax, 0.1) and np.allclose(ay, 0.1)
    # periodic: the first and last grid line are one line
    pred = np.array([[0.2, 0.0], [0.4, 0.0], [0.9, 0.0]])
    ov, ax, _ = mlp.setup_from_predictions(pred, 3, 1, 4, W.BC_PERIODIC)
    assert ov == [0, 1, 1]                              # rho = 0 -> at least 1
    assert np.allclose(ax, [0.55, 0.3, 0.65, 0.55])


def test_overlap_ratio_reproduces_paper_rules():
    for p in (4, 8, 12, 16):
        orders = level_orders(p)
        assert mlp.overlaps_from_ratio(1 / 8, p)[1:] == [max(1, math.ceil(q / 8)) for q in orders[1:]]
        assert mlp.overlaps_from_ratio(0.5, p)[1:] == [min(math.ceil(q / 2), q - 1) for q in orders[1:]]


def test_cycle_cost_reduces_to_paper_omega():
    # n_o = 0 on every level: m / n_p = 1 and W / r_bar must equal the paper's
    # omega_1 with c_s = sum of the relative level sizes and c_CG = 2
    for p in (4, 8, 16):
        orders = level_orders(p)
        L = len(orders) - 1
        cs = sum((q / p) ** 2 for q in orders[1:])
        for ns in (1, 2):
            W_ = mlp.cycle_cost(p, [0] * (L + 1), [ns] * (L + 1))
            assert W_ / 1.3 == pytest.approx(omega_k(1.3, p, 0, ns, cs=cs, ccg=2.0), rel=1e-14)
