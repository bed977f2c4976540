"""Wendland C2 smoothing kernel (section 3.3.1, Eq. 16-17) and the pair force of Eq. 15.

W(r, h) = alpha_d (1 - q/2)^4 (2q + 1) for 0 <= q <= 2, 0 beyond, with q = r/h.

Readings:
  * Eq. 16 calls q "the model dimension"; it is the normalised distance r/h
    (the support ends at q = 2, i.e. at r_c = 2h).
  * Eq. 17 prints alpha_3 = 21/(6 pi h^3). The kernel integrates to one over
    R^3 only with 21/(16 pi h^3); the printed 2-D constant 7/(4 pi h^2) is
    consistent with the same polynomial. We use 21/(16 pi h^3).
  * Eq. 15 with unit mass (Eq. 13) and a uniform target density has the
    constant prefactor p0/rho_t^2 + p0/rho_t^2; it is taken as 1. It cancels
    from the positions because the time step normalises by the largest
    acceleration.
"""
import math

import numpy as np


def alpha(h: float, d: int = 3) -> float:
    """Normalisation factor alpha_d of Eq. 17 (3-D value corrected, see module doc)."""
    if d == 2:
        return 7.0 / (4.0 * math.pi * h * h)
    if d == 3:
        return 21.0 / (16.0 * math.pi * h ** 3)
    raise ValueError(d)


def W(r, h, d: int = 3):
    """Eq. 16."""
    q = np.asarray(r, np.float64) / h
    t = np.clip(1.0 - 0.5 * q, 0.0, None)
    return alpha(h, d) * t ** 4 * (2.0 * q + 1.0)


def dW_dr(r, h, d: int = 3):
    """Derivative of Eq. 16 with respect to r: -(5 alpha / h) q (1 - q/2)^3."""
    q = np.asarray(r, np.float64) / h
    t = np.clip(1.0 - 0.5 * q, 0.0, None)
    return -(5.0 * alpha(h, d) / h) * q * t ** 3


def force_coef(h: float) -> float:
    """K such that -dW/dr * e_ij = K (1 - q/2)^3 (x_i - x_j)  (Eq. 15, prefactor 1)."""
    return 5.0 * alpha(h, 3) / (h * h)
