"""Central finite-difference weights for the second derivative.

The paper discretises the Laplacian with a high-order central finite
difference (Sec. 4: a nine-point formula, i.e. half-width p = 4).  The
weights c_m, m = -p..p, are the unique symmetric solution of the Taylor
(moment) system

    sum_m c_m m^k = 2 * delta_{k,2},   k = 0..2p,

solved here exactly in rational arithmetic.  f''(0) ~ h^-2 sum_m c_m f(m h).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np


def fd_weights_exact(p: int) -> List[Fraction]:
    """c_{-p..p} as exact fractions (Gaussian elimination on the Taylor system)."""
    if p < 1:
        raise ValueError("half-width must be >= 1")
    ms = list(range(-p, p + 1))
    n = 2 * p + 1
    a = [[Fraction(m) ** k for m in ms] + [Fraction(2 if k == 2 else 0)] for k in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        inv = 1 / a[col][col]
        a[col] = [x * inv for x in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [a[i][n] for i in range(n)]


def fd_weights(p: int) -> np.ndarray:
    """c_{-p..p} as float64 (index m + p)."""
    return np.array([float(c) for c in fd_weights_exact(p)])
