"""Learned Schwarz parameters (project extension, not in the paper): plain FP64
reference of every step the GPU performs.

Test infrastructure only: the solver library never calls this module.

The extension predicts, per element, a width scale alpha for the smoothed-sign
weights (Section 3.1: the transition zone of width delta_o around each
interface, Table 1) and an overlap ratio rho (the subdomain overlap n_o,l of
Section 4, chosen per level as ceil(rho p_l)) from local features of the mesh
and of the diffusivity nu (Section 4, variable diffusion).

Network: d_in -> 64 (tanh) -> 64 (tanh) -> d_out (logistic), parameters
packed as W1 (64 x d_in, row-major), b1, W2 (64 x 64), b2, W3 (d_out x 64), b3.
Loss: L = 1/(2n) sum_s sum_o (y_so - t_so)^2.  Optimiser: Adam with
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.

Features of element e (d_in = 8):
  0  log2(h_x / h_y)
  1  ln nu_bar_e (the GLL-quadrature element mean, as in the local solves)
  2-5  ln nu_bar of the left, right, lower, upper neighbour minus ln nu_bar_e
       (0 where the side is a Dirichlet boundary; periodic sides wrap)
  6  ln(max nu / min nu) over the element's nodes
  7  p / 32

Reduction of per-element predictions (alpha_e, q_e) to solver parameters (the
GPU kernels need one overlap per level and a width scale that is constant
along each grid line, which keeps the weights a partition of unity):
  alpha_e = min(max(alpha_e, 0.1), 1)
  alpha at a grid line = mean of alpha_e over the elements that touch the line
  rho = 0.5 * mean_e q_e
  n_o,l = ceil(rho p_l), clamped to [1, p_l - 1] and to p_l + 1 + 2 n_o,l <= 48

Cost of one MGCG iteration in units of one finest-level operator application
(the paper's omega measure, Section 4, generalised to an overlap per level):
  W = sum_{l>=1} (p_l / p_L)^2 [2 (m_l / n_p,l)^3 n_s,l + 1] + c_CG / 2
with m_l = p_l + 1 + 2 n_o,l, n_p,l = p_l + 1, n_s,l the smoothing steps of
level l and c_CG = 2; omega = W / r_bar is the cost per decade of residual
reduction.  For one n_o / n_p on all levels and c_s = sum_l 4^(l-L) this is
the paper's omega_1 formula.
"""
from __future__ import annotations

import math

import numpy as np

from .discretization import PERIODIC, Space, element_mean
from .multigrid import level_orders

WIDTH = 64
D_IN = 8
D_OUT = 2
ALPHA_MIN = 0.1
MAX_TILE = 48
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def n_params(d_in: int = D_IN, width: int = WIDTH, d_out: int = D_OUT) -> int:
    return width * d_in + width + width * width + width + d_out * width + d_out


def unpack(theta, d_in: int = D_IN, width: int = WIDTH, d_out: int = D_OUT):
    theta = np.asarray(theta, dtype=np.float64)
    sizes = [(width, d_in), (width,), (width, width), (width,), (d_out, width), (d_out,)]
    out, k = [], 0
    for s in sizes:
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    assert k == theta.size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X, d_in: int = D_IN, d_out: int = D_OUT):
    """Network output Y (n x d_out) and the hidden activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, d_in, WIDTH, d_out)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(X @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    Y = 1.0 / (1.0 + np.exp(-(H2 @ W3.T + b3)))
    return Y, (X, H1, H2)


def loss(theta, X, T, d_in: int = D_IN, d_out: int = D_OUT) -> float:
    Y, _ = forward(theta, X, d_in, d_out)
    return float(0.5 * np.sum((Y - np.asarray(T)) ** 2) / len(Y))


def gradient(theta, X, T, d_in: int = D_IN, d_out: int = D_OUT):
    """Loss and its gradient by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, d_in, WIDTH, d_out)
    Y, (X, H1, H2) = forward(theta, X, d_in, d_out)
    T = np.asarray(T, dtype=np.float64)
    n = len(Y)
    L = 0.5 * np.sum((Y - T) ** 2) / n
    dY = (Y - T) / n
    dZ3 = dY * Y * (1.0 - Y)               # logistic derivative
    gW3 = dZ3.T @ H2
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3) * (1.0 - H2 ** 2)     # tanh derivative
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (1.0 - H1 ** 2)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    return float(L), pack([gW1, gb1, gW2, gb2, gW3, gb3])


class Adam:
    """Adam (Kingma & Ba) with bias correction, FP64."""

    def __init__(self, theta):
        self.theta = np.array(theta, dtype=np.float64)
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0

    def step(self, g, lr: float):
        self.t += 1
        self.m = BETA1 * self.m + (1 - BETA1) * g
        self.v = BETA2 * self.v + (1 - BETA2) * g * g
        mh = self.m / (1 - BETA1 ** self.t)
        vh = self.v / (1 - BETA2 ** self.t)
        self.theta = self.theta - lr * mh / (np.sqrt(vh) + EPS)
        return self.theta


def element_features(xb, yb, p: int, bc: int, NU=None) -> np.ndarray:
    """(ny*nx) x 8 feature rows, element e = ey * nx + ex."""
    sp = Space(xb, yb, p, bc)
    nx, ny = sp.ax.n, sp.ay.n
    if NU is None:
        NU = np.ones(sp.shape)
    lnb = np.log(element_mean(sp, NU))     # (ny, nx)
    F = np.zeros((ny * nx, D_IN))
    per = bc == PERIODIC
    for ey in range(ny):
        for ex in range(nx):
            e = ey * nx + ex
            F[e, 0] = math.log2(sp.ax.h[ex] / sp.ay.h[ey])
            F[e, 1] = lnb[ey, ex]
            for k, (dy, dx) in enumerate(((0, -1), (0, 1), (-1, 0), (1, 0))):
                jy, jx = ey + dy, ex + dx
                if per:
                    jy, jx = jy % ny, jx % nx
                elif not (0 <= jy < ny and 0 <= jx < nx):
                    continue
                F[e, 2 + k] = lnb[jy, jx] - lnb[ey, ex]
            gy, gx = sp.element_nodes(ey, ex)
            Ne = NU[np.ix_(gy, gx)]
            F[e, 6] = math.log(Ne.max() / Ne.min())
            F[e, 7] = p / 32.0
    return F


def overlaps_from_ratio(rho: float, p: int):
    """n_o per level (entry 0 unused) for overlap ratio rho."""
    out = [0]
    for pl in level_orders(p)[1:]:
        n = math.ceil(rho * pl)
        n = min(max(n, 1), pl - 1, (MAX_TILE - 1 - pl) // 2)
        out.append(n)
    return out


def setup_from_predictions(pred, nx: int, ny: int, p: int, bc: int):
    """(overlaps per level, alpha per x grid line, alpha per y grid line)."""
    pred = np.asarray(pred, dtype=np.float64).reshape(ny, nx, 2)
    alpha = np.clip(pred[:, :, 0], ALPHA_MIN, 1.0)
    rho = 0.5 * float(np.mean(pred[:, :, 1]))
    ax = np.zeros(nx + 1)
    for i in range(nx + 1):
        cols = [c for c in (i - 1, i) if 0 <= c < nx]
        if bc == PERIODIC and i in (0, nx):
            cols = [nx - 1, 0]
        ax[i] = np.mean(alpha[:, cols])
    ay = np.zeros(ny + 1)
    for j in range(ny + 1):
        rows = [r for r in (j - 1, j) if 0 <= r < ny]
        if bc == PERIODIC and j in (0, ny):
            rows = [ny - 1, 0]
        ay[j] = np.mean(alpha[rows, :])
    return overlaps_from_ratio(rho, p), ax, ay


def cycle_cost(p: int, overlaps, ns, c_cg: float = 2.0) -> float:
    """W of one MGCG iteration in finest-operator units (module docstring);
    ns[l] = pre + post smoothing steps of level l."""
    orders = level_orders(p)
    W = c_cg / 2.0
    for l in range(1, len(orders)):
        pl = orders[l]
        m = pl + 1 + 2 * overlaps[l]
        W += (pl / p) ** 2 * (2.0 * (m / (pl + 1)) ** 3 * ns[l] + 1.0)
    return W
