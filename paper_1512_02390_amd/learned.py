"""Learned Schwarz parameters (project extension; the paper fixes them by hand).

Per element, a network predicts a width scale alpha for the smoothed-sign
weights (Section 3.1, Table 1: the transition zone of width delta_o around an
interface becomes alpha * delta_o) and an overlap ratio (Section 4 uses
n_o,l = ceil(p_l / 8); here n_o,l = ceil(rho p_l)).  Everything runs through
the library:

  1. training data: the solver sweeps (alpha, rho) on small patch meshes of
     uniform aspect ratio and random diffusivity, runs a few MGCG iterations
     for each candidate and keeps the candidate with the lowest cost per
     decade of residual reduction, omega = W / r_bar (W: work of one
     iteration in finest-operator units, see ``cycle_cost``); every element
     of the patch becomes one sample (its features, that label);
  2. training: the library's MLP kernels (forward, backward, Adam) on the GPU;
  3. inference: element features and the forward pass on the GPU; each
     element's prediction (alpha_e, rho_e) goes to the library either as its
     own parameters (sem_weights.elem_params: per-element overlap and
     transition width inside the Schwarz kernels, Shepard-normalised) or
     reduced to one overlap per level and one width scale per grid line
     (sem_learned_params); the paper's parameters are the fallback when the
     prediction is unusable or the learned solve fails.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import workloads as W
from .metrics import cycle_cost, level_orders, rbar  # noqa: F401  (re-exported)
from .sem import MLP, SemError, Solver, learned_params

ALPHAS = (0.25, 0.5, 0.75, 1.0)
RATIOS = (0.125, 0.25, 0.375, 0.5)
PATCH_AR = (1.0, 2.0, 4.0, 8.0, 16.0)
PATCH_SIGMA = (0.0, 0.5, 1.0)
PATCH_P = (12, 32)
PATCH_N = 8
SWEEP_ITERS = 6
SEED_SWEEP = 100


def overlaps_for(rho: float, p: int):
    """n_o per level for overlap ratio rho (the library's rule)."""
    ov, _, _ = learned_params(np.array([[1.0, 2.0 * rho]], dtype=np.float32), 1, 1, p,
                              W.BC_DIRICHLET)
    return ov


@dataclass
class Patch:
    ar: float
    sigma: float
    p: int
    seed: int

    def mesh(self):
        hy = 1.0 / PATCH_N
        return W.uniform_breaks(PATCH_N, PATCH_N * self.ar * hy), W.uniform_breaks(PATCH_N, 1.0)


def nodal_nu(xb, yb, p: int, bc: int, field):
    """Nodal diffusivity at the finest nodes (coordinates from the library)."""
    if field is None:
        return None
    probe = Solver(xb, yb, p, bc, 1, 1, 5)
    xc, yc = probe.node_coords()
    probe.close()
    return W.nodal(field.nu, xc, yc)


def schedule(L: int, kind: str = "mg11"):
    if kind == "mg10":
        return [1] * (L + 1), [0] * (L + 1)
    if kind == "mg11":
        return [1] * (L + 1), [1] * (L + 1)
    ns = [2 ** (L - l) for l in range(L + 1)]
    return ns, list(ns)


def sweep_patch(patch: Patch, kind: str = "mg11", alphas=ALPHAS, ratios=RATIOS):
    """Features of the patch's elements (device tensor) and the table of
    (alpha, rho, r_bar, omega) of every candidate; the label is the row of
    smallest omega."""
    import torch
    xb, yb = patch.mesh()
    bc = W.BC_DIRICHLET
    field = W.GaussianFieldNu(seed=patch.seed, ell=1.0, sigma=patch.sigma) if patch.sigma > 0 else None
    NU = nodal_nu(xb, yb, patch.p, bc, field)
    base = Solver(xb, yb, patch.p, bc, 1, 1, 5, nu=NU)
    feats = base.elem_features()
    shape = base.shape()
    base.close()
    fn = torch.tensor(W.random_nodal(shape, bc, W.SEED_RHS), dtype=torch.float64, device="cuda")
    u0 = torch.tensor(W.random_guess(shape, bc, W.SEED_U0), dtype=torch.float64, device="cuda")
    rows = []
    for rho in ratios:
        ov = overlaps_for(rho, patch.p)
        for a in alphas:
            s = Solver(xb, yb, patch.p, bc, 0, 1, 5, nu=NU, overlaps=ov,
                       alpha_x=np.full(len(xb), a), alpha_y=np.full(len(yb), a))
            b = s.zeros()
            s.mass(fn, b)
            ns1, ns2 = schedule(s.L, kind)
            u = u0.clone()
            try:
                _, hist, _ = s.pcg_solve(u, b, SWEEP_ITERS, 0.0, ns1, ns2)
                r = rbar(hist)
            except SemError:
                r = 0.0
            s.close()
            ns = [x + y for x, y in zip(ns1, ns2)]
            om = cycle_cost(patch.p, ov, ns) / r if r > 0 else math.inf
            rows.append((a, rho, r, om))
    return feats, rows


def label_of(rows):
    """Target (alpha, 2 rho) of the candidate with the smallest omega."""
    best = min(rows, key=lambda t: t[3])
    return best[0], 2.0 * best[1]


def make_dataset(patches, kind: str = "mg11"):
    """(X, T, records): X (n, 8) and T (n, 2) FP32 device tensors."""
    import torch
    xs, ts, recs = [], [], []
    for pt in patches:
        feats, rows = sweep_patch(pt, kind)
        a, q = label_of(rows)
        xs.append(feats)
        ts.append(torch.tensor([[a, q]] * feats.shape[0], dtype=torch.float32, device="cuda"))
        recs.append((pt, rows, (a, q)))
    return torch.cat(xs), torch.cat(ts), recs


def default_patches(ars=PATCH_AR, sigmas=PATCH_SIGMA, ps=PATCH_P):
    out, k = [], 0
    for p in ps:
        for ar in ars:
            for sg in sigmas:
                out.append(Patch(ar, sg, p, SEED_SWEEP + k))
                k += 1
    return out


def train(X, T, steps: int = 1500, lr: float = 3e-3, seed: int = W.SEED_MLP):
    """Full-batch Adam on the GPU; returns the network and the loss history
    (every 100 steps and the last)."""
    net = MLP(W.mlp_init(seed=seed))
    hist = []
    for k in range(steps):
        want = k % 100 == 0 or k == steps - 1
        l = net.train_step(X, T, lr, want_loss=want)
        if want:
            hist.append(l)
    return net, hist


def elem_params_of(pred) -> np.ndarray | None:
    """Per-element (alpha_e, rho_e) from network outputs (alpha, q = 2 rho):
    alpha clipped to [0.1, 1]; None when a prediction is not finite."""
    pred = np.asarray(pred, dtype=np.float64)
    if not np.all(np.isfinite(pred)):
        return None
    return np.stack([np.clip(pred[:, 0], 0.1, 1.0), np.maximum(0.5 * pred[:, 1], 0.0)], axis=1)


def predict(solver: Solver, net: MLP):
    """Per-element parameters (n_e, 2) for a problem, or None when the
    prediction is unusable (the caller then keeps the paper's parameters)."""
    pred = net.forward(solver.elem_features()).cpu().numpy()
    return elem_params_of(pred)


def solver_with_learned(xb, yb, p: int, bc: int, NU, net: MLP, precision: int = 0,
                        mode: str = "level"):
    """Solver with learned parameters, or the paper's (ceil(p_l/8), alpha = 1)
    when the prediction is unusable.  Returns (solver, per-element parameters
    (n_e, 2) or None).

    mode "element": every element keeps its own prediction (overlap and width
    per subdomain inside the Schwarz kernels, Shepard-normalised).
    mode "level": the predictions are reduced by the library
    (sem_learned_params) to one overlap per level (from the mean ratio) and
    one width scale per grid line -- on the variable-diffusion workloads this
    is the mode that lowers the iteration count (the network's smaller
    overlaps on the square elements cost iterations when kept per element)."""
    base = Solver(xb, yb, p, bc, 1, 1, 5, nu=NU)
    ep = predict(base, net)
    base.close()
    if ep is None:
        return Solver(xb, yb, p, bc, 1, 1, 5, nu=NU, precision=precision), None
    if mode == "element":
        return Solver(xb, yb, p, bc, 1, 1, 5, nu=NU, precision=precision, elem_params=ep), ep
    pred = np.stack([ep[:, 0], 2.0 * ep[:, 1]], axis=1)
    try:
        ov, ax, ay = learned_params(pred, len(xb) - 1, len(yb) - 1, p, bc)
    except SemError:
        return Solver(xb, yb, p, bc, 1, 1, 5, nu=NU, precision=precision), None
    s = Solver(xb, yb, p, bc, 0, 1, 5, nu=NU, precision=precision, overlaps=ov,
               alpha_x=ax, alpha_y=ay)
    return s, ep
