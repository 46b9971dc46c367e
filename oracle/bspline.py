"""ORACLE (test infrastructure): uniform B-spline temporal basis.

N^{beta,d}(t) = sum_{kappa=0}^{d+1} w^{kappa,d} ((t - t_{kappa+beta})/dt)_+^d   (eq. decompose)
w^{kappa,d}   = (d+1) / prod_{k=0, k!=kappa}^{d+1} (k - kappa)                  (eq. w, Table 1)
"""
from fractions import Fraction

import numpy as np


def w_exact(kappa: int, d: int) -> Fraction:
    p = Fraction(1)
    for k in range(d + 2):
        if k != kappa:
            p *= (k - kappa)
    return Fraction(d + 1) / p


def weights(d: int) -> np.ndarray:
    return np.array([float(w_exact(k, d)) for k in range(d + 2)])


def basis(beta: int, d: int, t, dt: float = 1.0):
    """N^{beta,d}(t) with knots t_i = i*dt (eq. decompose)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    for k, wk in enumerate(weights(d)):
        out += wk * np.clip((t - (k + beta) * dt) / dt, 0.0, None) ** d
    return out
