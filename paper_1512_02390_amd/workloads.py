"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the solver: no GLL points, no operators, no
mass scaling.  It only produces element break points, random arrays and
analytic functions (exact solutions, sources, diffusivities) that each side then
evaluates at its own node coordinates.

Workloads follow the paper's test protocol (Section 4): a random initial guess
in [0, 1], sources evaluated analytically from an exact solution, Cartesian
meshes of rectangular elements.  The named configurations are:

  c1  Poisson, [0,1]^2, 4x4 uniform elements, p=4, Dirichlet, manufactured sine.
  c2  Poisson, [0,1]^2, 64x64 uniform elements, p=8, Dirichlet, random RHS.
  c3  Poisson, [0,1]^2, 128x128 uniform elements, p=16, Dirichlet, random RHS.
  c4  Variable diffusion, 32x32 elements, x widths growing geometrically to an
      aspect ratio of 16, p=12, nu = exp(g) with g a Gaussian random field
      (sigma = 1, correlation length 1.0: with the x-stretched elements a
      shorter correlation length leaves nu unresolved by the element means
      and the method diverges).
  c5  As c4 on 48x48 elements with p=32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_DIRICHLET = 0
BC_PERIODIC = 1

# Seeds: initial guess, right-hand side, random field, MLP init.
SEED_U0 = 0
SEED_RHS = 1
SEED_GRF = 2
SEED_MLP = 3


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_breaks(n: int, length: float) -> np.ndarray:
    """n equal elements on [0, length]."""
    return np.linspace(0.0, length, n + 1)


def geometric_breaks(n: int, h0: float, ratio: float) -> np.ndarray:
    """Element widths h0 * ratio**(i/(n-1)), i = 0..n-1, starting at 0."""
    if n == 1:
        return np.array([0.0, h0])
    widths = h0 * ratio ** (np.arange(n) / (n - 1))
    return np.concatenate([[0.0], np.cumsum(widths)])


def node_array_shape(nx: int, ny: int, p: int, bc: int) -> tuple[int, int]:
    """(rows, cols) of the nodal array: Dirichlet keeps the boundary nodes."""
    if bc == BC_DIRICHLET:
        return ny * p + 1, nx * p + 1
    return ny * p, nx * p


def zero_dirichlet_boundary(a: np.ndarray, bc: int) -> np.ndarray:
    if bc == BC_DIRICHLET:
        a = a.copy()
        a[0, :] = 0.0
        a[-1, :] = 0.0
        a[:, 0] = 0.0
        a[:, -1] = 0.0
    return a


def random_guess(shape, bc: int, seed: int = SEED_U0) -> np.ndarray:
    """Initial guess drawn i.i.d. from U[0, 1] on the unknowns."""
    return zero_dirichlet_boundary(rng(seed).uniform(0.0, 1.0, size=shape), bc)


def random_nodal(shape, bc: int, seed: int = SEED_RHS) -> np.ndarray:
    """Nodal source values drawn i.i.d. from U[-1, 1] on the unknowns."""
    return zero_dirichlet_boundary(rng(seed).uniform(-1.0, 1.0, size=shape), bc)


# ----------------------------------------------------------------------------
# Analytic fields.  Every callable takes broadcastable coordinate arrays.
# ----------------------------------------------------------------------------

@dataclass
class SineSolution:
    """u = sin(kx x) sin(ky y) with kx = pi*ax, ky = pi*ay."""
    ax: float = 1.0
    ay: float = 1.0

    @property
    def kx(self):
        return math.pi * self.ax

    @property
    def ky(self):
        return math.pi * self.ay

    def u(self, x, y):
        return np.sin(self.kx * x) * np.sin(self.ky * y)

    def grad(self, x, y):
        return (self.kx * np.cos(self.kx * x) * np.sin(self.ky * y),
                self.ky * np.sin(self.kx * x) * np.cos(self.ky * y))

    def laplacian(self, x, y):
        return -(self.kx ** 2 + self.ky ** 2) * self.u(x, y)


@dataclass
class ConstantNu:
    c: float = 1.0

    def nu(self, x, y):
        return np.full(np.broadcast(x, y).shape, self.c)

    def grad(self, x, y):
        z = np.zeros(np.broadcast(x, y).shape)
        return z, z


@dataclass
class PaperNu:
    """nu = 1 + amp sin(2 pi (x - s)) sin(2 pi (y - s)), the paper's variable
    diffusivity test (Section 4, variable diffusion)."""
    amp: float = 0.9
    s: float = 0.2

    def nu(self, x, y):
        k = 2 * math.pi
        return 1.0 + self.amp * np.sin(k * (x - self.s)) * np.sin(k * (y - self.s))

    def grad(self, x, y):
        k = 2 * math.pi
        return (self.amp * k * np.cos(k * (x - self.s)) * np.sin(k * (y - self.s)),
                self.amp * k * np.sin(k * (x - self.s)) * np.cos(k * (y - self.s)))


@dataclass
class GaussianFieldNu:
    """nu = exp(g), g a stationary Gaussian field with variance sigma^2 and
    squared-exponential covariance exp(-|d|^2 / (2 ell^2)), represented by K
    random Fourier features: g = sqrt(2/K) sum_k cos(w_k . x + phi_k) with
    w_k ~ N(0, ell^-2 I) and phi_k ~ U[0, 2 pi).  Analytic everywhere, so every
    multigrid level can evaluate it at its own nodes."""
    seed: int = SEED_GRF
    ell: float = 1.0
    sigma: float = 1.0
    K: int = 1024
    omega: np.ndarray = field(init=False, repr=False)
    phase: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.omega = g.normal(0.0, 1.0 / self.ell, size=(self.K, 2))
        self.phase = g.uniform(0.0, 2 * math.pi, size=self.K)

    def _arg(self, x, y):
        x = np.asarray(x, dtype=np.float64)[..., None]
        y = np.asarray(y, dtype=np.float64)[..., None]
        return x * self.omega[:, 0] + y * self.omega[:, 1] + self.phase

    def g(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if x.ndim == 2 and y.ndim == 2 and x.shape[0] == 1 and y.shape[1] == 1:
            # tensor grid (row of x, column of y): cos(a + b) = cos a cos b -
            # sin a sin b per feature, summed over the features by two matrix
            # products instead of one cosine per node and feature
            a = x[0][:, None] * self.omega[:, 0] + self.phase     # (nx, K)
            b = y[:, 0][:, None] * self.omega[:, 1]               # (ny, K)
            s = np.cos(b) @ np.cos(a).T - np.sin(b) @ np.sin(a).T
            return self.sigma * math.sqrt(2.0 / self.K) * s
        return self.sigma * math.sqrt(2.0 / self.K) * np.cos(self._arg(x, y)).sum(-1)

    def nu(self, x, y):
        return np.exp(self.g(x, y))

    def grad(self, x, y):
        s = -self.sigma * math.sqrt(2.0 / self.K) * np.sin(self._arg(x, y))
        gx = (s * self.omega[:, 0]).sum(-1)
        gy = (s * self.omega[:, 1]).sum(-1)
        n = self.nu(x, y)
        return n * gx, n * gy


def diffusion_source(sol: SineSolution, nu, x, y):
    """f = -(nu lap u + grad nu . grad u) for -div(nu grad u) = f."""
    nx, ny = nu.grad(x, y)
    ux, uy = sol.grad(x, y)
    return -(nu.nu(x, y) * sol.laplacian(x, y) + nx * ux + ny * uy)


def nodal(fn, xc: np.ndarray, yc: np.ndarray) -> np.ndarray:
    """Evaluate fn(x, y) on the tensor grid (rows = y, cols = x)."""
    return fn(xc[None, :], yc[:, None])


# ----------------------------------------------------------------------------
# Named configurations (sizes only).
# ----------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    nx: int
    ny: int
    p: int
    bc: int
    xb: np.ndarray
    yb: np.ndarray
    overlap_rule: int      # 0 fixed, 1 ceil(p_l/8), 2 floor(p_l/8), 3 ceil(p_l/2)
    n_o: int               # used when overlap_rule == 0
    variable_nu: bool
    description: str
    overlaps: list | None = None   # explicit n_o per level (entry 0 unused)


OVERLAP_FIXED, OVERLAP_CEIL8, OVERLAP_FLOOR8, OVERLAP_CEIL2 = 0, 1, 2, 3


def config(name: str, n_o: int = 1) -> Config:
    name = name.lower()
    if name == "c1":
        return Config("c1", 4, 4, 4, BC_DIRICHLET, uniform_breaks(4, 1.0), uniform_breaks(4, 1.0),
                      OVERLAP_FIXED, 1, False,
                      "Poisson [0,1]^2, 4x4 elements, p=4, Dirichlet, sine RHS")
    if name == "c2":
        return Config("c2", 64, 64, 8, BC_DIRICHLET, uniform_breaks(64, 1.0), uniform_breaks(64, 1.0),
                      OVERLAP_FIXED, n_o, False,
                      f"Poisson [0,1]^2, 64x64 elements, p=8, Dirichlet, n_o={n_o}")
    if name == "c3":
        return Config("c3", 128, 128, 16, BC_DIRICHLET, uniform_breaks(128, 1.0),
                      uniform_breaks(128, 1.0), OVERLAP_CEIL8, 0, False,
                      "Poisson [0,1]^2, 128x128 elements, p=16, Dirichlet, ceil(p_l/8)")
    if name in ("c4", "c5"):
        n, p = (32, 12) if name == "c4" else (48, 32)
        h = 1.0 / n
        return Config(name, n, n, p, BC_DIRICHLET, geometric_breaks(n, h, 16.0),
                      uniform_breaks(n, 1.0), OVERLAP_CEIL8, 0, True,
                      f"variable nu=exp(GRF), {n}x{n} elements stretched to AR 16, p={p}")
    raise ValueError(name)


# ----------------------------------------------------------------------------
# Network initialisation for the learned-parameter extension (random numbers
# only; the network arithmetic lives on each side).
# ----------------------------------------------------------------------------

def mlp_init(d_in: int = 8, width: int = 64, d_out: int = 2, seed: int = SEED_MLP) -> np.ndarray:
    """Flat parameter vector W1, b1, W2, b2, W3, b3 (weights row-major, out x in):
    weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero.  Values are
    rounded to float32 so that FP32 and FP64 consumers start from the same
    numbers."""
    g = rng(seed)
    parts = []
    for fi, fo in ((d_in, width), (width, width), (width, d_out)):
        b = math.sqrt(6.0 / (fi + fo))
        parts.append(g.uniform(-b, b, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
