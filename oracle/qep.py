"""Dense solution of the quadratic eigenvalue problem and its checks.

The set the Sakurai-Sugiura method computes is, by definition (paper Eqs. 4
and 5), every lambda with det P(lambda) = 0 and lambda_min < |lambda| <
1/lambda_min, together with its eigenvector.  This module computes that set
directly: lambda P(lambda) = H- + lambda (H0 - E) + lambda^2 H+ is linearised
to the 2N x 2N companion pencil

    A v = lambda B v,   A = [[0, I], [-H-, -(H0 - E)]],   B = [[I, 0], [0, H+]],

with v = [x; lambda x], and the pencil is solved with LAPACK's QZ
(scipy.linalg.eig).  The left eigenvector w of the pencil gives y = w[N:],
which satisfies y^H P(lambda) = 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .fd import fd_weights


@dataclasses.dataclass
class QepResult:
    lam: np.ndarray        # [m] complex eigenvalues inside the annulus
    x: np.ndarray          # [N, m] right eigenvectors, unit 2-norm
    y: np.ndarray          # [N, m] left eigenvectors (y^H P(lam) = 0), unit 2-norm
    all_lam: np.ndarray    # every finite eigenvalue of the pencil


def P_dense(h0, hp, hm, E, z):
    return (h0 - E * np.eye(h0.shape[0])) + z * hp + hm / z


def solve_dense(h0, hp, hm, E, lambda_min, left=True) -> QepResult:
    n = h0.shape[0]
    eye = np.eye(n)
    zero = np.zeros((n, n))
    A = np.block([[zero, eye], [-hm, -(h0 - E * eye)]])
    B = np.block([[eye, zero], [zero, hp]])
    if left:
        ab, wl, vr = sla.eig(A, B, left=True, right=True, homogeneous_eigvals=True)
    else:
        ab, vr = sla.eig(A, B, left=False, right=True, homogeneous_eigvals=True)
        wl = None
    alpha, beta = ab
    finite = np.abs(beta) > 1e-13 * np.abs(alpha)
    lam_all = np.full(alpha.shape, np.inf + 0j)
    lam_all[finite] = alpha[finite] / beta[finite]
    keep = finite & (np.abs(lam_all) > lambda_min) & (np.abs(lam_all) < 1.0 / lambda_min)
    lam = lam_all[keep]
    x = vr[:n, keep]
    x = x / np.linalg.norm(x, axis=0, keepdims=True)
    if wl is not None:
        y = wl[n:, keep]
        y = y / np.linalg.norm(y, axis=0, keepdims=True)
    else:
        y = np.zeros_like(x)
    order = np.lexsort((np.angle(lam), np.abs(np.log(np.abs(lam)))))
    return QepResult(lam[order], x[:, order], y[:, order], lam_all[finite])


def residuals(h0, hp, hm, E, lam, x):
    """||P(lambda) x||_2 / ||x||_2 for each pair."""
    out = np.empty(len(lam))
    for i, l in enumerate(lam):
        out[i] = np.linalg.norm(P_dense(h0, hp, hm, E, l) @ x[:, i]) / np.linalg.norm(x[:, i])
    return out


def dispersion_1d(p: int, h: float, theta: np.ndarray) -> np.ndarray:
    """Kinetic energy of e^{i theta n} under -1/2 FD Laplacian on one axis."""
    c = fd_weights(p)
    acc = c[p] * np.ones_like(theta)
    for m in range(1, p + 1):
        acc = acc + 2.0 * c[p + m] * np.cos(m * theta)
    return -0.5 * acc / (h * h)


def free_electron_lambdas(nx, ny, nz, h, p, E) -> np.ndarray:
    """All finite nonzero Bloch factors of the V = 0 crystal.

    Plane waves e^{i(theta_x ix + theta_y iy)} mu^{iz} diagonalise the free
    finite-difference operator.  For each transverse pair the z factor mu
    solves  eps_perp - 1/2 h^-2 sum_m c_m mu^m = E, a degree-2p polynomial
    after multiplying by mu^p, and the cell factor is lambda = mu^{nz}.
    """
    c = fd_weights(p)
    tx = 2 * np.pi * np.arange(nx) / nx
    ty = 2 * np.pi * np.arange(ny) / ny
    ex = dispersion_1d(p, h, tx)
    ey = dispersion_1d(p, h, ty)
    out = []
    for a in ex:
        for b in ey:
            coef = c.astype(np.complex128).copy()        # powers mu^{m+p}, m=-p..p
            coef[p] += 2.0 * h * h * (E - a - b)
            roots = np.roots(coef[::-1])                 # highest power first
            out.append(roots ** nz)
    return np.concatenate(out)


def lambda_to_k(lam, cell_length: float) -> np.ndarray:
    """Complex wave number of each Bloch factor (Sec. 2: lambda = exp(i k a), a the cell
    length): k = log(lambda) / (i a) with the principal complex logarithm."""
    lam = np.asarray(lam, dtype=np.complex128)
    return np.log(lam) / (1j * cell_length)


def in_annulus(lam, lambda_min):
    lam = np.asarray(lam)
    return lam[(np.abs(lam) > lambda_min) & (np.abs(lam) < 1.0 / lambda_min)]


def hk_distance(h0, hp, hm, E, lam):
    """min |eig(H(k)) - E| for a unimodular lambda = e^{ik a} (paper Sec. 4.1)."""
    hk = h0 + lam * hp + np.conj(lam) * hm
    hk = 0.5 * (hk + hk.conj().T)
    ev = np.linalg.eigvalsh(hk)
    return float(np.min(np.abs(ev - E)))


def bands_dense(h0, hp, hm, k, cell_length, n_bands):
    """The lowest n_bands eigenvalues of the Hermitian H(k) = H0 + e^{ika} H+ + e^{-ika} H-
    (the conventional band structure at real k; Sec. 2, Sec. 4.1), by LAPACK."""
    lam = np.exp(1j * k * cell_length)
    hk = h0 + lam * hp + np.conj(lam) * hm
    hk = 0.5 * (hk + hk.conj().T)
    return np.linalg.eigvalsh(hk)[:n_bands]


def free_electron_bands(nx, ny, nz, h, p, k, n_bands):
    """Closed form of the lowest bands of the free finite-difference crystal (V = 0, no
    projectors): plane waves with transverse phases 2 pi n / N and phase (k a + 2 pi n_z) / nz
    per grid step along z have the eigenvalues eps_perp + eps_z of the 1-D dispersions."""
    a = nz * h
    ex = dispersion_1d(p, h, 2 * np.pi * np.arange(nx) / nx)
    ey = dispersion_1d(p, h, 2 * np.pi * np.arange(ny) / ny)
    ez = dispersion_1d(p, h, (k * a + 2 * np.pi * np.arange(nz)) / nz)
    all_ = (ex[:, None, None] + ey[None, :, None] + ez[None, None, :]).reshape(-1)
    return np.sort(all_)[:n_bands]


def match_sets(a, b):
    """Greedy nearest matching of two eigenvalue sets; returns max relative gap."""
    a = list(np.asarray(a))
    b = list(np.asarray(b))
    if len(a) != len(b):
        return np.inf
    worst = 0.0
    for v in a:
        j = int(np.argmin([abs(v - w) for w in b]))
        worst = max(worst, abs(v - b[j]) / abs(v))
        b.pop(j)
    return worst
