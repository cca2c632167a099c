"""Sakurai-Sugiura steps in the paper's order, with plain dense algebra.

Sec. 3.1 (Eqs. 6-8, Algorithm 1) and the ring contour of Sec. 3.2:
  1. solve P(z_j) Y_j = V at every quadrature point of both circles;
  2. moments  S_k = sum_j w_j^(1) (z_j^(1))^k Y_j^(1) - sum_j w_j^(2) (z_j^(2))^k Y_j^(2)
     and mu_k = V^H S_k;
  3. block Hankel T_ij = mu_{i+j}, T<_ij = mu_{i+j+1} (0-based i, j < M),
     truncated SVD T ~ U1 S1 W1^H with the rank threshold delta, the reduced
     problem U1^H T< W1 S1^{-1} phi = tau phi and psi = S W1 S1^{-1} phi with
     S = [S_0 ... S_{M-1}].
The Rayleigh-Ritz variant projects the QEP onto orth(S W1) and solves the
small QEP densely.  ``bicg`` is the BiCG iteration that solves a system and
its dual at once (Sec. 3.2, Eq. 11): the dual of P(z) is P(z)^H = P(1/conj z).
``half_stop_iteration`` is the load-balancing stop of Sec. 3.3.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import qep as _qep


def quadrature(lambda_min: float, n_q: int):
    """Nodes and weights on the outer (1) and inner (2) circle.

    theta_j = 2 pi (j - 1/2) / n_q, z^(1) = e^{i theta}/lambda_min,
    z^(2) = lambda_min e^{i theta}.  The weight is the trapezoid rule of
    (1/2 pi i) \\oint dz on a circle of radius rho: dz = i z d theta, so
    w_j = z_j / n_q.  (The printed weight e^{i theta_j}/n_q omits the radius;
    with it the inner circle's contribution would not cancel the poles inside
    it.)  Returns (z1, w1, z2, w2).
    """
    j = np.arange(1, n_q + 1)
    theta = 2 * np.pi * (j - 0.5) / n_q
    e = np.exp(1j * theta)
    z1 = e / lambda_min
    z2 = lambda_min * e
    return z1, z1 / n_q, z2, z2 / n_q


def moments(Y1, Y2, z1, w1, z2, w2, n_k):
    """S_k for k < n_k from per-node solutions Y[j] of shape [N, L]."""
    out = []
    for k in range(n_k):
        s = sum(w1[j] * z1[j] ** k * Y1[j] for j in range(len(z1)))
        s = s - sum(w2[j] * z2[j] ** k * Y2[j] for j in range(len(z2)))
        out.append(s)
    return out


def hankel(mu, M):
    L = mu[0].shape[0]
    T = np.zeros((L * M, L * M), dtype=np.complex128)
    Tl = np.zeros_like(T)
    for i in range(M):
        for j in range(M):
            T[i * L:(i + 1) * L, j * L:(j + 1) * L] = mu[i + j]
            Tl[i * L:(i + 1) * L, j * L:(j + 1) * L] = mu[i + j + 1]
    return T, Tl


@dataclasses.dataclass
class SSResult:
    lam_hankel: np.ndarray
    psi_hankel: np.ndarray
    lam_rr: np.ndarray
    psi_rr: np.ndarray
    sigma: np.ndarray
    rank: int
    mu: list
    S: list


def ss_dense(H, E, V, lambda_min, n_q, M, delta=1e-10):
    """Algorithm 1 on the ring contour, Step 1 by dense LU solves.

    H is an ``oracle.ham.Hamiltonian``; V is [L, N] (rows are right-hand sides).
    """
    h0, hp, hm = H.blocks_dense()
    Vc = np.ascontiguousarray(V.T)                      # [N, L]
    z1, w1, z2, w2 = quadrature(lambda_min, n_q)
    Y1 = [np.linalg.solve(_qep.P_dense(h0, hp, hm, E, z), Vc) for z in z1]
    Y2 = [np.linalg.solve(_qep.P_dense(h0, hp, hm, E, z), Vc) for z in z2]
    S = moments(Y1, Y2, z1, w1, z2, w2, 2 * M)
    mu = [Vc.conj().T @ s for s in S]
    res = extract(mu, S[:M], M, delta)
    lam_rr, psi_rr = rayleigh_ritz(h0, hp, hm, E, S[:M], res[3], res[2], lambda_min)
    return SSResult(res[0], res[1], lam_rr, psi_rr, res[4], res[2], mu, S)


def extract(mu, S_low, M, delta):
    """Hankel SVD truncation and the reduced standard eigenproblem."""
    T, Tl = hankel(mu, M)
    U, s, Wh = np.linalg.svd(T)
    rank = int(np.sum(s > delta * s[0]))
    U1 = U[:, :rank]
    W1 = Wh.conj().T[:, :rank]
    s1 = s[:rank]
    red = U1.conj().T @ Tl @ W1 / s1[None, :]
    tau, phi = np.linalg.eig(red)
    Sm = np.concatenate(S_low, axis=1)                  # [N, L*M]
    psi = Sm @ (W1 / s1[None, :]) @ phi
    psi = psi / np.linalg.norm(psi, axis=0, keepdims=True)
    return tau, psi, rank, W1, s


def rayleigh_ritz(h0, hp, hm, E, S_low, W1, rank, lambda_min):
    """Project the QEP onto Q = orth(S W1) and solve the small QEP densely."""
    Sm = np.concatenate(S_low, axis=1)
    Q, _ = np.linalg.qr(Sm @ W1[:, :rank])
    a0 = Q.conj().T @ (h0 @ Q)
    ap = Q.conj().T @ (hp @ Q)
    am = Q.conj().T @ (hm @ Q)
    r = _qep.solve_dense(a0, ap, am, E, lambda_min, left=False)
    psi = Q @ r.x
    psi = psi / np.linalg.norm(psi, axis=0, keepdims=True)
    return r.lam, psi


def bicg(apply, apply_dual, b, b_dual, tol=1e-10, max_iter=10000, fixed_iters=None, history=None):
    """BiCG for A x = b together with the dual A^H xt = b_dual.

    apply(v) = A v, apply_dual(v) = A^H v.  Scalars alpha = (rt^H r)/(pt^H A p),
    beta = (rt_new^H r_new)/(rt^H r); the dual recurrences use conj(alpha),
    conj(beta).  Stops when both relative residuals are below tol, or after
    ``fixed_iters`` iterations when that is given.  Returns (x, xt, iters,
    relres, relres_dual).  If ``history`` is a list, the pair of relative
    residuals after every iteration is appended to it.
    """
    x = np.zeros_like(b)
    xt = np.zeros_like(b_dual)
    r = b.copy()
    rt = b_dual.copy()
    p = r.copy()
    pt = rt.copy()
    nb = np.linalg.norm(b)
    nbt = np.linalg.norm(b_dual)
    rho = np.vdot(rt, r)
    it = 0
    limit = fixed_iters if fixed_iters is not None else max_iter
    while it < limit:
        q = apply(p)
        qt = apply_dual(pt)
        sigma = np.vdot(pt, q)
        alpha = rho / sigma
        x = x + alpha * p
        xt = xt + np.conj(alpha) * pt
        r = r - alpha * q
        rt = rt - np.conj(alpha) * qt
        it += 1
        rr = np.linalg.norm(r) / nb
        rrt = np.linalg.norm(rt) / nbt
        if history is not None:
            history.append((rr, rrt))
        if fixed_iters is None and rr < tol and rrt < tol:
            break
        rho_new = np.vdot(rt, r)
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
        pt = rt + np.conj(beta) * pt
    return x, xt, it, np.linalg.norm(r) / nb, np.linalg.norm(rt) / nbt


def block_bicg(apply, apply_dual, B, tol=1e-10, max_iter=10000):
    """Block BiCG (O'Leary's block form of the BiCG of ``bicg``) for A X = B with the dual
    A^H Xt = B, B of shape [N, L]: the scalars become L x L matrices,

        alpha = (Pt^H A P)^-1 (Rt^H R),   alphat = (Pt^H A P)^-H (Rt^H R)^H
        X += P alpha,  Xt += Pt alphat,   R -= A P alpha,  Rt -= A^H Pt alphat
        beta = (Rt^H R)^-1 (Rt^H R)_new,  betat = (Rt^H R)^-H (Rt^H R)_new^H
        P = R + P beta,  Pt = Rt + Pt betat

    (L = 1 gives ``bicg``).  Stops when every column's primal and dual relative residual is
    below tol.  apply / apply_dual act on [N, L] blocks.  Returns (X, Xt, iters, relres
    [L], relres_dual [L])."""
    X = np.zeros_like(B)
    Xt = np.zeros_like(B)
    R = B.copy()
    Rt = B.copy()
    P = R.copy()
    Pt = Rt.copy()
    nb = np.linalg.norm(B, axis=0)
    rho = Rt.conj().T @ R
    it = 0
    while it < max_iter:
        Q = apply(P)
        Qt = apply_dual(Pt)
        sigma = Pt.conj().T @ Q
        alpha = np.linalg.solve(sigma, rho)
        alphat = np.linalg.solve(sigma.conj().T, rho.conj().T)
        X = X + P @ alpha
        Xt = Xt + Pt @ alphat
        R = R - Q @ alpha
        Rt = Rt - Qt @ alphat
        it += 1
        rr = np.linalg.norm(R, axis=0) / nb
        rrt = np.linalg.norm(Rt, axis=0) / nb
        if np.all(rr < tol) and np.all(rrt < tol):
            break
        rho_new = Rt.conj().T @ R
        beta = np.linalg.solve(rho, rho_new)
        betat = np.linalg.solve(rho.conj().T, rho_new.conj().T)
        rho = rho_new
        P = R + P @ beta
        Pt = Rt + Pt @ betat
    return X, Xt, it, np.linalg.norm(R, axis=0) / nb, np.linalg.norm(Rt, axis=0) / nb


def half_stop_iteration(node_iters):
    """Iteration at which the load-balancing rule of Sec. 3.3 stops every solve.

    The solves at all quadrature points advance together, one BiCG iteration each per
    step, and all stop as soon as more than half of the points have converged.  A point
    has converged when every right-hand side at it has, so its count is the largest over
    its right-hand sides: ``node_iters[j]``.  More than half of n points are done after
    the (n // 2 + 1)-th smallest count.  The iterate a run holds under the rule is its
    iterate after min(own count, this iteration) steps (the solves do not interact).
    """
    counts = sorted(int(c) for c in node_iters)
    if not counts:
        raise ValueError("no quadrature points")
    return counts[len(counts) // 2]
