"""Shape functions and the nonuniform weight function (Section 3.1).

The 1-D weight of a subdomain is
    w(xi) = 1/2 [ phi((xi + 1)/delta) - phi((xi - 1)/delta) ]      (eq. weight function)
with xi the standard coordinate of the element extended beyond [-1, 1] and
delta the overlap width.  phi equals a polynomial phi^ on [-1, 1] and sgn(x)
outside (eq. shape function).  Table 1 lists phi^ for the linear, cubic,
quintic and 7th-order cases, the top hat (phi^ = sgn) and the arithmetic mean
(phi^ = 0).

Reading of the paper: the polynomial degree in the defining conditions is
kappa (the text's "degree i" is a misprint).  For odd kappa the conditions
phi^(+-1) = +-1 and vanishing derivatives up to order (kappa-1)/2 at +-1 are met
by the normalised integral of (1 - t^2)^((kappa-1)/2); Table 1's polynomials are
used verbatim for kappa <= 7 and the tests check that both forms agree.
"""
from __future__ import annotations

import math

import numpy as np

# wf identifiers (negative values are the two non-polynomial cases of Table 1,
# and the multiplicative method of Algorithm 1, which uses no weights)
WF_TOPHAT = -1
WF_ARITH = -2
WF_MULT = -3

TABLE1 = {
    1: lambda x: x,
    3: lambda x: (3 * x - x ** 3) / 2,
    5: lambda x: (15 * x - 10 * x ** 3 + 3 * x ** 5) / 8,
    7: lambda x: (35 * x - 35 * x ** 3 + 21 * x ** 5 - 5 * x ** 7) / 16,
}


def phi_hat_integral(kappa: int, x):
    """phi^_kappa(x) = int_0^x (1-t^2)^q dt / int_0^1 (1-t^2)^q dt, q = (kappa-1)/2,
    expanded with the binomial theorem."""
    q = (kappa - 1) // 2
    x = np.asarray(x, dtype=np.float64)
    num = np.zeros_like(x)
    den = 0.0
    for k in range(q + 1):
        c = math.comb(q, k) * (-1) ** k / (2 * k + 1)
        num = num + c * x ** (2 * k + 1)
        den += c
    return num / den


def phi(kappa: int, x):
    """Shape function phi_kappa on the real line (eq. shape function)."""
    x = np.asarray(x, dtype=np.float64)
    if kappa == WF_TOPHAT:
        return np.sign(x)
    if kappa == WF_ARITH:
        # phi^ = 0 on the open interval; sgn outside.  Used only as a check of
        # the counting definition (see schwarz.counting_weights).
        return np.where(np.abs(x) < 1.0, 0.0, np.sign(x))
    inner = TABLE1[kappa](x) if kappa in TABLE1 else phi_hat_integral(kappa, x)
    return np.where(np.abs(x) <= 1.0, inner, np.sign(x))


def weight(kappa: int, xi, delta_left: float, delta_right: float,
           left_saturated: bool = False, right_saturated: bool = False):
    """w(xi) = 1/2 [phi((xi+1)/delta_l) - phi((xi-1)/delta_r)].

    With equal widths this is the paper's weight function.  A saturated side
    (a Dirichlet boundary, where no neighbouring subdomain exists) takes its
    limiting value, phi = +1 on the left and -1 on the right, so that the
    weights still sum to one at every unknown."""
    xi = np.asarray(xi, dtype=np.float64)
    left = np.ones_like(xi) if left_saturated else phi(kappa, (xi + 1.0) / delta_left)
    right = -np.ones_like(xi) if right_saturated else phi(kappa, (xi - 1.0) / delta_right)
    return 0.5 * (left - right)


def overlap_width(xi_gll: np.ndarray, n_o: int) -> float:
    """delta_o = xi_{n_o+1} + 1 (Section 3.1)."""
    return float(xi_gll[n_o + 1] + 1.0)
