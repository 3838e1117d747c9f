"""Convergence and cost measures (Section 4).

r_bar = (1/n) log10(||r^(0)|| / ||r^(n)||), Euclidean norm; n_10 is the number
of cycles for a 10^10 reduction, the smallest integer >= 10 / r_bar.
omega_k = (k / r_bar) W_cyc / W_op with W_op = 2 n_p^3 n_e and
W_cyc = [4 (1 + 2 n_o/n_p)^3 c_s n_s + 2 c_s + c_CG] n_p^3 n_e, n_p = p + 1,
c_s = 4/3 (V-cycle) or 2 (variable V-cycle), c_CG = 2 for MGCG and 0 for MG.

Reading: the printed tables agree with this formula only after an extra
factor n_p / p; both values are reported (``omega_k`` and ``omega_k_tables``).
"""
from __future__ import annotations

import math


def rbar(res_hist, n=None) -> float:
    n = len(res_hist) - 1 if n is None else n
    return math.log10(res_hist[0] / res_hist[n]) / n


def n10(r: float) -> int:
    return math.ceil(10.0 / r - 1e-12)


def omega_k(r: float, p: int, n_o: int, n_s: int = 1, cs: float = 4.0 / 3.0,
            ccg: float = 0.0, k: int = 1) -> float:
    n_p = p + 1
    w_cyc = 4.0 * (1.0 + 2.0 * n_o / n_p) ** 3 * cs * n_s + 2.0 * cs + ccg
    return (k / r) * w_cyc / 2.0


def omega_k_tables(r: float, p: int, n_o: int, n_s: int = 1, cs: float = 4.0 / 3.0,
                   ccg: float = 0.0, k: int = 1) -> float:
    return omega_k(r, p, n_o, n_s, cs, ccg, k) * (p + 1) / p
