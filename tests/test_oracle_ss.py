"""Pins of the oracle's Sakurai-Sugiura steps (paper Sec. 3, Algorithm 1).

* quadrature: for the scalar P(z) = z - a the trapezoid moments on the ring
  equal a^k F(a) with F(a) = 1/(1+(a/rho1)^N) - 1/(1+(a/rho2)^N) for k < N,
  a closed form obtained by expanding 1/(z - a) in a geometric series (the
  shifted nodes satisfy z_j^N = -rho^N);
* brute force: a diagonal QEP whose roots are known in closed form;
* the whole dense SS pipeline against QZ on the smallest configuration;
* BiCG and its dual against a dense LU solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ham, qep, ss


@pytest.mark.parametrize("a", [0.3, 0.9 + 0.2j, -1.5j, 1.9, 2.6, 0.7 * np.exp(2j)])
def test_quadrature_filter_closed_form(a):
    lmin, N = 0.5, 32
    z1, w1, z2, w2 = ss.quadrature(lmin, N)
    rho1, rho2 = 1 / lmin, lmin
    F = 1 / (1 + (a / rho1) ** N) - 1 / (1 + (a / rho2) ** N)
    for k in range(0, N):
        sk = np.sum(w1 * z1 ** k / (z1 - a)) - np.sum(w2 * z2 ** k / (z2 - a))
        # rounding of a sum whose largest terms are ~ rho1^k
        assert abs(sk - a ** k * F) <= 1e-13 + 1e-15 * N * rho1 ** k


def test_quadrature_nodes():
    z1, w1, z2, w2 = ss.quadrature(0.5, 32)
    np.testing.assert_allclose(np.abs(z1), 2.0)
    np.testing.assert_allclose(np.abs(z2), 0.5)
    np.testing.assert_allclose(z2, 1 / np.conj(z1), rtol=1e-15)
    np.testing.assert_allclose(z1 ** 32, -(2.0 ** 32), rtol=1e-12)


class _Diag:
    """A decoupled QEP: every diagonal entry is a scalar quadratic."""

    def __init__(self, d0, dp):
        self.h0, self.hp = np.diag(d0), np.diag(dp)

    def blocks_dense(self):
        return self.h0, self.hp, self.hp.T


def test_ss_diagonal_qep_brute_force():
    rng = np.random.default_rng(11)
    n = 40
    d0 = rng.uniform(-3, 3, n)
    dp = rng.uniform(0.5, 1.5, n)
    E = 0.2
    # roots of (d0 - E) + lam dp + dp / lam = 0
    b = d0 - E
    roots = np.concatenate([(-b + np.sqrt(b * b - 4 * dp * dp + 0j)) / (2 * dp),
                            (-b - np.sqrt(b * b - 4 * dp * dp + 0j)) / (2 * dp)])
    want = qep.in_annulus(roots, 0.5)
    # keep away from the contour so the filter does not matter
    assert np.min(np.abs(np.abs(np.log(np.abs(roots))) - np.log(2))) > 0.05
    V = W.make_rhs(n, 8, 5)
    r = ss.ss_dense(_Diag(d0, dp), E, V, 0.5, 32, 8)
    got = qep.in_annulus(r.lam_rr, 0.5)
    assert len(got) == len(want) > 4
    assert qep.match_sets(got, want) < 1e-10


@pytest.fixture(scope="module")
def cfg1_e1():
    s = W.config(1).systems[0]
    H = ham.build(s)
    h0, hp, hm = H.blocks_dense()
    return H, qep.solve_dense(h0, hp, hm, 1.0, 0.5, left=False)


def test_ss_matches_qz_cfg1(cfg1_e1):
    H, ref = cfg1_e1
    V = W.make_rhs(H.n, 8, 3001)
    r = ss.ss_dense(H, 1.0, V, 0.5, 32, 8)
    assert r.rank < 64
    assert qep.match_sets(qep.in_annulus(r.lam_rr, 0.5), ref.lam) < 1e-10
    assert qep.match_sets(qep.in_annulus(r.lam_hankel, 0.5), ref.lam) < 1e-6
    # lambda does not depend on the random block V
    r2 = ss.ss_dense(H, 1.0, W.make_rhs(H.n, 8, 999), 0.5, 32, 8)
    assert qep.match_sets(qep.in_annulus(r2.lam_rr, 0.5), ref.lam) < 1e-10


def test_bicg_primal_and_dual_match_lu():
    s = W.tiny(with_proj=True, fd_order=8)
    H = ham.build(s)
    h0, hp, hm = H.blocks_dense()
    z1, _, z2, _ = ss.quadrature(0.5, 32)
    v = W.make_rhs(s.n, 1, 3)[0]
    for j in (0, 7, 20):
        x, xt, it, rr, rrt = ss.bicg(lambda u: H.apply(z1[j], u, 0.7),
                                     lambda u: H.apply(1 / np.conj(z1[j]), u, 0.7), v, v)
        assert rr < 1e-10 and rrt < 1e-10
        np.testing.assert_allclose(x, np.linalg.solve(qep.P_dense(h0, hp, hm, 0.7, z1[j]), v), atol=1e-8)
        np.testing.assert_allclose(xt, np.linalg.solve(qep.P_dense(h0, hp, hm, 0.7, z2[j]), v), atol=1e-8)


@pytest.mark.parametrize("tol,bar", [(1e-10, 1e-8), (1e-12, 1e-10)])
def test_eigen_residual_follows_solve_tolerance(tol, bar):
    # Algorithm 1 with Step 1 done by BiCG to a relative residual tol: the moments carry
    # the solve error, so the Rayleigh-Ritz pairs reach ||P(lambda) psi|| ~ 10-50 tol
    # (QZ gives the count); the bars this sets are the ones the device path is held to
    sysw = W.tiny(with_proj=True, fd_order=8)
    H = ham.build(sysw)
    h0, hp, hm = H.blocks_dense()
    E, L, M = 4.0, 8, 8
    n = h0.shape[0]
    Vc = np.ascontiguousarray(W.make_rhs(n, L, 7).T)
    z1, w1, z2, w2 = ss.quadrature(0.5, 32)
    Y1, Y2 = [], []
    for z in z1:
        A = qep.P_dense(h0, hp, hm, E, z)
        AH = A.conj().T
        a = np.zeros((n, L), complex)
        b = np.zeros((n, L), complex)
        for l in range(L):
            out = ss.bicg(lambda v: A @ v, lambda v: AH @ v, Vc[:, l], Vc[:, l], tol=tol, max_iter=20000)
            a[:, l], b[:, l] = out[0], out[1]
        Y1.append(a)
        Y2.append(b)
    S = ss.moments(Y1, Y2, z1, w1, z2, w2, 2 * M)
    mu = [Vc.conj().T @ s for s in S]
    res = ss.extract(mu, S[:M], M, 1e-10)
    lam, psi = ss.rayleigh_ritz(h0, hp, hm, E, S[:M], res[3], res[2], 0.5)
    ref = qep.solve_dense(h0, hp, hm, E, 0.5, left=False).lam
    assert len(lam) == len(ref) and qep.match_sets(lam, ref) <= 1e-8
    r = qep.residuals(h0, hp, hm, E, lam, psi)
    assert r.max() <= bar
    assert r.max() >= 1e-3 * bar   # the residual is set by the solves, not by rounding


@pytest.mark.parametrize("real_v", [True, False])
def test_mirrored_nodes_of_real_sources(real_v):
    """The blocks are real, so P(conj z) = conj P(z).  With real V the solution at the
    mirrored node conj z_j (node n_q-1-j, theta -> 2 pi - theta) is conj Y_j on both circles,
    the moments S_k are real, and summing 2 Re(w z^k Y) over the nodes with 0 < theta < pi
    gives S_k (what the device path does with conj_nodes).  With complex V the mirror
    identity fails (the negative control)."""
    sysw = W.tiny(with_proj=True, fd_order=4)
    h0, hp, hm = ham.build(sysw).blocks_dense()
    for b in (h0, hp, hm):
        assert np.max(np.abs(np.imag(b))) == 0.0
    E, nq, L = 4.0, 8, 2
    rng = np.random.default_rng(5)
    V = rng.standard_normal((sysw.n, L))
    if not real_v:
        V = V + 1j * rng.standard_normal((sysw.n, L))
    z1, w1, z2, w2 = ss.quadrature(0.5, nq)
    Y1 = [np.linalg.solve(qep.P_dense(h0, hp, hm, E, z), V) for z in z1]
    Y2 = [np.linalg.solve(qep.P_dense(h0, hp, hm, E, z), V) for z in z2]
    scale = max(np.max(np.abs(y)) for y in Y1 + Y2)
    mirror_err = max(max(np.max(np.abs(Y[nq - 1 - j] - np.conj(Y[j]))) for j in range(nq)) for Y in (Y1, Y2))
    np.testing.assert_allclose(z1[::-1], np.conj(z1), rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(w1[::-1], np.conj(w1), rtol=1e-15, atol=1e-15)
    S = ss.moments(Y1, Y2, z1, w1, z2, w2, 6)
    if real_v:
        assert mirror_err <= 1e-12 * scale
        h = nq // 2
        for k, sk in enumerate(S):
            half = sum(w1[j] * z1[j] ** k * Y1[j] - w2[j] * z2[j] ** k * Y2[j] for j in range(h))
            assert np.max(np.abs(sk.imag)) <= 1e-12 * np.max(np.abs(sk))
            np.testing.assert_allclose(2 * half.real, sk.real, rtol=0, atol=1e-12 * np.max(np.abs(sk)))
    else:
        assert mirror_err > 1e-3 * scale


def test_half_stop_iteration_is_the_first_step_with_more_than_half_done():
    # brute force of the rule's definition: step the solves together and stop at the first
    # step after which more than half of the points have converged
    assert ss.half_stop_iteration([5, 9, 3, 7]) == 7          # 3 of 4 done after step 7
    assert ss.half_stop_iteration([1, 2, 3, 4, 5]) == 3       # 3 of 5 done after step 3
    assert ss.half_stop_iteration([4]) == 4
    assert ss.half_stop_iteration([6, 6, 6, 2]) == 6          # ties: 2 of 4 is not more than half
    rng = np.random.default_rng(11)
    for _ in range(200):
        counts = rng.integers(1, 40, size=int(rng.integers(1, 33)))
        t = 0
        while 2 * int(np.sum(counts <= t)) <= len(counts):
            t += 1
        assert ss.half_stop_iteration(counts) == t


def test_half_stop_rule_keeps_the_slowest_point_within_1e_8():
    # Sec. 4.1: with BiCG to 1e-10 at every point of config 1 (8x8x12), stopping all solves
    # once more than half of the points converged leaves the slowest runs below 1e-8, and
    # the eigenvalues still match the dense QEP
    sysw = W.config(1).systems[0]
    H = ham.build(sysw)
    h0, hp, hm = H.blocks_dense()
    E, L, M, nq = 0.3, 8, 8, 32
    n = h0.shape[0]
    Vc = np.ascontiguousarray(W.make_rhs(n, L, 7).T)
    z1, w1, z2, w2 = ss.quadrature(0.5, nq)
    A = [qep.P_dense(h0, hp, hm, E, z) for z in z1]
    AH = [np.ascontiguousarray(a.conj().T) for a in A]
    full = [[ss.bicg(lambda v: a @ v, lambda v: ah @ v, Vc[:, l], Vc[:, l], tol=1e-10)
             for l in range(L)] for a, ah in zip(A, AH)]
    its = np.array([[out[2] for out in row] for row in full])
    T = ss.half_stop_iteration(its.max(axis=1))
    assert T < its.max()   # the rule stops some runs early
    Y1, Y2, worst = [], [], 0.0
    for j, a in enumerate(A):
        y1 = np.zeros((n, L), complex)
        y2 = np.zeros((n, L), complex)
        for l in range(L):
            out = full[j][l]
            if its[j, l] > T:
                out = ss.bicg(lambda v: a @ v, lambda v: AH[j] @ v, Vc[:, l], Vc[:, l], fixed_iters=T)
            y1[:, l], y2[:, l] = out[0], out[1]
            worst = max(worst, out[3], out[4])
        Y1.append(y1)
        Y2.append(y2)
    assert 1e-10 <= worst <= 1e-8
    S = ss.moments(Y1, Y2, z1, w1, z2, w2, 2 * M)
    mu = [Vc.conj().T @ s for s in S]
    res = ss.extract(mu, S[:M], M, 1e-10)
    lam, psi = ss.rayleigh_ritz(h0, hp, hm, E, S[:M], res[3], res[2], 0.5)
    ref = qep.solve_dense(h0, hp, hm, E, 0.5, left=False).lam
    assert len(lam) == len(ref) and qep.match_sets(lam, ref) <= 1e-8
    assert qep.residuals(h0, hp, hm, E, lam, psi).max() <= 1e-8


def test_block_bicg_matches_lu_and_reduces_to_bicg():
    # the oracle's block BiCG (O'Leary's recurrences with L x L matrices) against the
    # definition of the result, LU solves of P(z) X = V and P(z)^H Xt = V; with one column it
    # is the scalar BiCG, iterate for iterate; a wrong transpose in either dual formula (alphat,
    # betat) breaks the dual solve, a wrong order of the L x L products the primal one
    sysw = W.tiny(with_proj=True, fd_order=8)
    h0, hp, hm = ham.build(sysw).blocks_dense()
    z1, _, _, _ = ss.quadrature(0.5, 32)
    B = W.make_rhs(sysw.n, 8, 3).T.copy()
    for j in (0, 7):
        A = qep.P_dense(h0, hp, hm, 4.0, z1[j])
        Ad = qep.P_dense(h0, hp, hm, 4.0, 1 / np.conj(z1[j]))
        X, Xt, it, rr, rrt = ss.block_bicg(lambda P: A @ P, lambda P: Ad @ P, B, tol=1e-11)
        assert np.all(rr < 1e-11) and np.all(rrt < 1e-11)
        nb = np.linalg.norm(B, axis=0)
        assert np.max(np.linalg.norm(B - A @ X, axis=0) / nb) <= 1e-10
        assert np.max(np.linalg.norm(B - Ad @ Xt, axis=0) / nb) <= 1e-10
        ref = np.linalg.solve(A, B)
        assert np.abs(X - ref).max() <= 1e-8 * np.abs(ref).max()
        its = [ss.bicg(lambda v: A @ v, lambda v: Ad @ v, B[:, l], B[:, l], tol=1e-11)[2] for l in range(8)]
        assert it < min(its)   # the block Krylov space grows 8 directions per iteration
        # one column: the iterates of the scalar recurrences (compared after 30 steps, before
        # the rounding differences of the two codes grow)
        x1, xt1, it1, _, _ = ss.block_bicg(lambda P: A @ P, lambda P: Ad @ P, B[:, :1], max_iter=30)
        x0, xt0, it0, _, _ = ss.bicg(lambda v: A @ v, lambda v: Ad @ v, B[:, 0], B[:, 0], fixed_iters=30)
        assert it1 == it0 == 30
        assert np.abs(x1[:, 0] - x0).max() <= 1e-11 * np.abs(x0).max()
        assert np.abs(xt1[:, 0] - xt0).max() <= 1e-11 * np.abs(xt0).max()
