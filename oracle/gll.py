"""Gauss-Lobatto-Legendre points, weights and Lagrange-basis operators.

Section 2 (eq. ansatz): the element basis is the Lagrange polynomials through
the GLL points {xi_i}, i = 0..p, on the standard region [-1, 1].  The 1-D
stiffness and mass matrices are the standard SEM ones, L^ = D^T W D and
M^ = W with W = diag(GLL weights); the mass is the GLL-quadrature (diagonal)
mass, and L^ is exact because its integrand has degree 2p-2.
"""
from __future__ import annotations

import math

import numpy as np


def legendre(n: int, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev, p_cur = np.ones_like(x), x.copy()
    d_prev, d_cur = np.zeros_like(x), np.ones_like(x)
    if n == 0:
        return p_prev, d_prev
    for k in range(2, n + 1):
        p_next = ((2 * k - 1) * x * p_cur - (k - 1) * p_prev) / k
        d_next = d_prev + (2 * k - 1) * p_cur
        p_prev, p_cur = p_cur, p_next
        d_prev, d_cur = d_cur, d_next
    return p_cur, d_cur


def gll(p: int):
    """GLL points xi_0 = -1 < ... < xi_p = 1 (ends plus the roots of P_p')
    and weights 2 / (p (p+1) P_p(xi_i)^2)."""
    if p < 1:
        raise ValueError("p >= 1")
    x = -np.cos(math.pi * np.arange(p + 1) / p)
    for _ in range(100):
        P, dP = legendre(p, x[1:-1])
        # Legendre ODE: (1 - x^2) P'' = 2 x P' - p (p+1) P
        d2P = (2 * x[1:-1] * dP - p * (p + 1) * P) / (1 - x[1:-1] ** 2)
        step = dP / d2P
        x[1:-1] -= step
        if np.all(np.abs(step) < 1e-16):
            break
    x[0], x[-1] = -1.0, 1.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def derivative_matrix(xi: np.ndarray) -> np.ndarray:
    """D[i, j] = l_j'(xi_i) for the Lagrange basis through xi (barycentric form)."""
    n = len(xi)
    lam = np.array([1.0 / np.prod([xi[j] - xi[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (xi[i] - xi[j])
        D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
    return D


def lagrange_matrix(xi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """E[q, j] = l_j(x_q), the Lagrange basis through xi evaluated at x."""
    x = np.asarray(x, dtype=np.float64)
    E = np.ones((len(x), len(xi)))
    for j in range(len(xi)):
        for k in range(len(xi)):
            if k != j:
                E[:, j] *= (x - xi[k]) / (xi[j] - xi[k])
    return E


def element_matrices(p: int):
    """Reference stiffness L^ = D^T W D and diagonal mass M^ = W on [-1, 1]."""
    xi, w = gll(p)
    D = derivative_matrix(xi)
    Lhat = D.T @ np.diag(w) @ D
    return Lhat, w.copy(), xi, w, D
