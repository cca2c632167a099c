"""Pins of the dense QEP oracle (paper Eqs. 4-5).

* closed form: with V = 0 and no projectors, plane waves diagonalise the
  operator and every Bloch factor is mu^{nz} for a root mu of a degree-2p
  polynomial (independent of the companion pencil and of QZ);
* pairing: P(lambda)^H = P(1/conj(lambda)) (paper Sec. 3.2) makes the set
  closed under lambda -> 1/conj(lambda); real symmetric blocks add conj;
* residual ||P(lambda) x|| / ||x|| <= 1e-10;
* propagating modes: for |lambda| = 1, E is an eigenvalue of the Hermitian
  H(k) = H0 + lambda H+ + conj(lambda) H- (the paper's accuracy test, Sec. 4.1).
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
