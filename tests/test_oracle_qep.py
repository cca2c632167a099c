"""Pins of the dense QEP oracle (paper Eqs. 4-5).

* closed form: with V = 0 and no projectors, plane waves diagonalise the
  operator and every Bloch factor is mu^{nz} for a root mu of a degree-2p
  polynomial (independent of the companion pencil and of QZ);
* pairing: P(lambda)^H = P(1/conj(lambda)) (paper Sec. 3.2) makes the set
  closed under lambda -> 1/conj(lambda); real symmetric blocks add conj;
* residual ||P(lambda) x|| / ||x|| <= 1e-10;
* propagating modes: for |lambda| = 1, E is an eigenvalue of the Hermitian
  H(k) = H0 + lambda H+ + conj(lambda) H- (the paper's accuracy test, Sec. 4.1);
* k of lambda = exp(i k a): inverse of the exponential on the strip
  -pi/a < Re k <= pi/a, decaying states (|lambda| < 1) have Im k > 0, and on a
  free chain the propagating k lie on the finite-difference band.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ham, qep


@pytest.fixture(scope="module")
def free_cfg1():
    s = W.free_system(8, 8, 12, 0.4, 4)
    return ham.build(s).blocks_dense()


@pytest.mark.parametrize("E,count", [(0.3, 2), (1.915, 10)])
def test_closed_form_free_electron(free_cfg1, E, count):
    h0, hp, hm = free_cfg1
    r = qep.solve_dense(h0, hp, hm, E, 0.5, left=False)
    cf = qep.in_annulus(qep.free_electron_lambdas(8, 8, 12, 0.4, 2, E), 0.5)
    assert len(r.lam) == len(cf) == count
    assert qep.match_sets(r.lam, cf) < 1e-12
    # the wider spectrum (all finite eigenvalues away from 0 and infinity) agrees too
    wide = lambda v: v[(np.abs(v) > 0.05) & (np.abs(v) < 20)]
    assert qep.match_sets(wide(r.all_lam), wide(qep.free_electron_lambdas(8, 8, 12, 0.4, 2, E))) < 1e-10


def test_closed_form_counts_second_threshold():
    # E = 1.915 lies just below the first transverse threshold eps_perp(1,0)
    eps10 = qep.dispersion_1d(2, 0.4, np.array([2 * np.pi / 8]))[0] + qep.dispersion_1d(2, 0.4, np.array([0.0]))[0]
    assert abs(eps10 - 1.91994) < 1e-4
    cf = qep.in_annulus(qep.free_electron_lambdas(8, 8, 12, 0.4, 2, 1.915), 0.5)
    mags = np.sort(np.abs(cf))
    np.testing.assert_allclose(mags[:4], 0.6205, atol=1e-4)
    np.testing.assert_allclose(mags[-4:], 1.6117, atol=1e-4)
    assert np.sum(np.abs(np.abs(cf) - 1) < 1e-12) == 2


@pytest.fixture(scope="module")
def tiny_e4():
    s = W.tiny(with_proj=True, fd_order=8)
    h0, hp, hm = ham.build(s).blocks_dense()
    return (h0, hp, hm), qep.solve_dense(h0, hp, hm, 4.0, 0.5)


def _check_invariants(blocks, E, r):
    h0, hp, hm = blocks
    assert len(r.lam) > 0
    assert qep.residuals(h0, hp, hm, E, r.lam, r.x).max() <= 1e-10
    # pairing lambda <-> 1/conj(lambda), and conj for real symmetric blocks
    assert qep.match_sets(r.lam, 1 / np.conj(r.lam)) < 1e-10
    assert qep.match_sets(r.lam, np.conj(r.lam)) < 1e-10
    # left vectors: y^H P(lambda) = 0
    for i, l in enumerate(r.lam):
        assert np.linalg.norm(r.y[:, i].conj() @ qep.P_dense(h0, hp, hm, E, l)) < 1e-10
    uni = [l for l in r.lam if abs(abs(l) - 1) < 1e-9]
    for l in uni:
        assert qep.hk_distance(h0, hp, hm, E, l) < 1e-10
    return uni


def test_invariants_tiny_with_projectors(tiny_e4):
    blocks, r = tiny_e4
    uni = _check_invariants(blocks, 4.0, r)
    assert len(r.lam) == 10 and len(uni) == 6


def test_invariants_cfg1():
    w = W.config(1)
    s = w.systems[0]
    h0, hp, hm = ham.build(s).blocks_dense()
    r = qep.solve_dense(h0, hp, hm, 1.0, 0.5)
    uni = _check_invariants((h0, hp, hm), 1.0, r)
    assert len(r.lam) == 6 and len(uni) == 4


def test_annulus_is_strict():
    lam = np.array([0.5, 0.5000001, 2.0, 1.9999999, 1.0])
    got = qep.in_annulus(lam, 0.5)
    assert list(got) == [0.5000001, 1.9999999, 1.0]


def test_lambda_to_k_inverts_the_bloch_factor():
    rng = np.random.default_rng(4)
    a = 4.8
    k = rng.uniform(-np.pi / a, np.pi / a, 200) * 0.999 + 1j * rng.uniform(-1.5, 1.5, 200)
    lam = np.exp(1j * k * a)
    np.testing.assert_allclose(qep.lambda_to_k(lam, a), k, rtol=0, atol=1e-12)
    # decaying along +z (|lambda| < 1) means Im k > 0; |lambda| = 1 means real k
    got = qep.lambda_to_k(np.array([0.5, 0.5j, 2.0, 1j]), a)
    assert got[0].imag > 0 and got[1].imag > 0 and got[2].imag < 0 and got[3].imag == 0
    assert abs(got[1].real - np.pi / 2 / a) < 1e-15 and abs(got[3].real - np.pi / 2 / a) < 1e-15


@pytest.mark.parametrize("E", [0.4, 1.3])
def test_lambda_to_k_of_a_free_chain_lies_on_the_band(E):
    # one transverse mode (nx = ny = 1): mu = exp(i theta) with E = eps(theta) and
    # lambda = mu^nz, so k h equals theta up to a multiple of 2 pi / nz
    nz, h, p = 12, 0.4, 4
    lam = qep.free_electron_lambdas(1, 1, nz, h, p, E)
    prop = lam[np.abs(np.abs(lam) - 1) < 1e-10]
    assert len(prop) == 2
    k = qep.lambda_to_k(prop, nz * h)
    assert np.max(np.abs(k.imag)) < 1e-10
    assert abs(k[0].real + k[1].real) < 1e-10      # +k and -k
    shifts = 2 * np.pi * np.arange(nz) / nz
    for kk in k.real:
        eps = qep.dispersion_1d(p, h, kk * h + shifts)
        assert np.min(np.abs(eps - E)) < 1e-10


def test_match_sets_negative_controls():
    # the comparator behind every eigenvalue parity test: equal sets (in any order) give 0,
    # a set with one value moved gives that value's relative gap, sets of different sizes
    # give inf, and a duplicate that hides a missing value is caught (greedy one-to-one
    # matching, not nearest-neighbour distances)
    a = np.array([0.6 + 0.2j, 1.5 - 0.3j, -0.8 + 0.6j, 0.55j])
    assert qep.match_sets(a, a[::-1]) == 0.0
    b = a.copy()
    b[2] = -0.8 + 0.61j
    assert abs(qep.match_sets(a, b) - 0.01 / abs(a[2])) < 1e-12
    assert qep.match_sets(a, a[:3]) == np.inf
    assert qep.match_sets(a[:3], a) == np.inf
    dup = np.array([a[0], a[0], a[2], a[3]])
    assert qep.match_sets(a, dup) > 0.5
    assert qep.match_sets(a, a * (1 + 1e-9)) <= 1.0000001e-9


@pytest.mark.parametrize("k_frac", [0.0, 0.37, -0.81])
def test_bands_dense_free_electron_closed_form(k_frac):
    # the oracle's conventional bands (eigvalsh of the assembled Hermitian H(k)) against the
    # closed form of the free finite-difference crystal: transverse phases 2 pi n / N and z
    # phase (k a + 2 pi n_z) / nz per grid step; a sign error in the Bloch phase of H+ or H-
    # moves every band with n_z != 0
    sysw = W.free_system(4, 5, 6, 0.45, 4)
    h0, hp, hm = ham.build(sysw).blocks_dense()
    a = sysw.nz * sysw.h
    k = k_frac * np.pi / a
    got = qep.bands_dense(h0, hp, hm, k, a, 40)
    want = qep.free_electron_bands(4, 5, 6, 0.45, 2, k, 40)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
