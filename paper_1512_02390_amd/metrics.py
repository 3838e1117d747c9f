"""Convergence measures of Section 4 on the library's residual histories.

r_bar = (1/n) log10(||r_0|| / ||r_n||) over n iterations; n_10 = the number of
iterations for a 10^10 reduction, the smallest integer >= 10 / r_bar; the
cost per decade omega = W / r_bar with W the work of one iteration in units
of one finest-level operator application (``cycle_cost``).
"""
from __future__ import annotations

import math

import numpy as np


def level_orders(p: int):
    """p_l for l = 0..L: p_L = p, p_{l-1} = ceil(p_l / 2) down to 1."""
    ps = [p]
    while ps[-1] > 1:
        ps.append((ps[-1] + 1) // 2)
    return ps[::-1]


def rbar(hist) -> float:
    n = len(hist) - 1
    if n < 1 or not (hist[-1] > 0) or not np.all(np.isfinite(hist)):
        return 0.0
    return math.log10(hist[0] / hist[-1]) / n


def n10(r: float) -> int:
    return math.ceil(10.0 / r - 1e-12) if r > 0 else 0


def cycle_cost(p: int, overlaps, ns, c_cg: float = 2.0) -> float:
    """Work of one MGCG iteration in units of one finest-level operator
    application: sum over smoothed levels of the relative level size times
    (2 (m_l / n_p,l)^3 smoothing steps + 1 residual), plus c_CG / 2 -- the
    paper's omega cost generalised to one overlap per level (ns[l] = pre +
    post smoothing steps of level l; c_CG = 0 for a plain V-cycle)."""
    orders = level_orders(p)
    w = c_cg / 2.0
    for l in range(1, len(orders)):
        pl = orders[l]
        m = pl + 1 + 2 * overlaps[l]
        w += (pl / p) ** 2 * (2.0 * (m / (pl + 1)) ** 3 * ns[l] + 1.0)
    return w
