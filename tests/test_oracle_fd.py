"""Pins of the oracle's finite-difference weights (the Laplacian of paper Sec. 4)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.fd import fd_weights, fd_weights_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_second_derivative_central.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        toks = line.split()
        out[int(toks[0])] = [Fraction(t) for t in toks[1:]]
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_weights_match_published_table(p):
    c = fd_weights_exact(p)
    g = _golden()[p]
    assert c[p:] == g                      # c_0..c_p
    assert c[:p + 1] == g[::-1]            # symmetric


@pytest.mark.parametrize("p", [1, 2, 4])
def test_exact_on_polynomials(p):
    # f''(0) exact for x^k, k <= 2p+1 (odd degrees by symmetry)
    c = fd_weights(p)
    m = np.arange(-p, p + 1)
    for k in range(0, 2 * p + 2):
        got = np.sum(c * m.astype(float) ** k)
        want = 2.0 if k == 2 else 0.0
        assert abs(got - want) < 1e-9 * max(1, p ** k)
    # and not exact one degree higher (the order is exactly 2p)
    assert abs(np.sum(c * m.astype(float) ** (2 * p + 2))) > 1e-6


def test_order_of_accuracy_on_cosine():
    # error of the FD second derivative of cos(x) scales like h^{2p}
    for p in (2, 4):
        c = fd_weights(p)
        m = np.arange(-p, p + 1)
        errs = []
        for h in (0.2, 0.1):
            approx = np.sum(c * np.cos(m * h)) / h ** 2
            errs.append(abs(approx + 1.0))
        rate = np.log2(errs[0] / errs[1])
        assert abs(rate - 2 * p) < 0.2
