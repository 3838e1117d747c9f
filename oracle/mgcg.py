"""Inexact multigrid-preconditioned conjugate gradients (Section 3.3, Algorithm 4).

Reading of the paper: the beta line of the printed algorithm uses q; the text
states the Polak-Ribiere formula, which is beta = z^T (r - r_old) / delta, and
that is what is implemented.  r_old starts at zero as printed, so the first
beta equals the Fletcher-Reeves value.  The stopping threshold is relative:
||r||_2 <= rtol ||r_0||_2 with r_0 = f - A u on entry.  For a singular
(periodic) system the right side is projected onto the range (mean removed).
"""
from __future__ import annotations

import numpy as np


def mgcg(mg, U, F, imax: int, rtol: float, ns1=None, ns2=None, precond=None):
    """Returns (u, residual-norm history, iterations).  ``precond(r)`` replaces
    the V-cycle when given (used by the tests with a fixed SPD preconditioner)."""
    L = mg.L
    sp = mg.spaces[L]
    F = np.array(F, dtype=np.float64)
    if mg.bc == 1:
        F = np.where(sp.mask, F - F[sp.mask].mean(), 0.0)
    M = precond if precond is not None else (
        lambda r: mg.vcycle(np.zeros(sp.shape), r, ns1, ns2))
    U = np.array(U, dtype=np.float64)
    r_old = np.zeros(sp.shape)
    r = mg.residual(L, U, F)
    hist = [np.linalg.norm(r[sp.mask])]
    p = M(r)
    delta = np.vdot(p, r)
    it = 0
    for it in range(1, imax + 1):
        q = mg.op(L, p)
        alpha = delta / np.vdot(p, q)
        U = U + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r[sp.mask]))
        if hist[-1] <= rtol * hist[0]:
            break
        z = M(r)
        beta = np.vdot(z, r - r_old) / delta
        p = z + beta * p
        delta = np.vdot(z, r)
        r_old = r
    return U, np.array(hist), it


def textbook_pcg(A, b, x0, Minv, imax: int, rtol: float):
    """Standard PCG with Fletcher-Reeves beta for a fixed SPD preconditioner,
    on dense vectors.  Used only to pin ``mgcg`` in the tests."""
    x = x0.copy()
    r = b - A @ x
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    r0 = np.linalg.norm(r)
    xs = [x.copy()]
    for _ in range(imax):
        Ap = A @ p
        a = rz / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        xs.append(x.copy())
        if np.linalg.norm(r) <= rtol * r0:
            break
        z = Minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return xs
