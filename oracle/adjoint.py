"""Eigenvalue derivatives with respect to the local potential.

For a simple eigenvalue lambda with P(lambda) x = 0 and y^H P(lambda) = 0,
differentiating P(lambda(V); V) x = 0 and multiplying by y^H gives

    d lambda / d V(r) = - conj(y(r)) x(r) / (y^H P'(lambda) x),
    P'(lambda) = H+ - lambda^{-2} H-,

because V(r) enters P only through the diagonal of H0.  The chain rule to
Gaussian amplitudes A_a with V = sum_a A_a g_a is a sum over the grid.
Because P(lambda)^H = P(1/conj(lambda)) (paper Sec. 3.2), y is also the
right eigenvector of the pair partner 1/conj(lambda).
"""
from __future__ import annotations

import numpy as np


def dlambda_dv(hp, hm, lam, x, y):
    """[N] complex gradient of one eigenvalue; x, y from ``qep.solve_dense``."""
    dp = hp - hm / (lam * lam)
    den = np.vdot(y, dp @ x)
    return -np.conj(y) * x / den


def dlambda_damp(g, grad_v):
    """Chain to amplitudes: g is [n_atoms, N] (unit Gaussians), grad_v [N]."""
    return g @ grad_v
