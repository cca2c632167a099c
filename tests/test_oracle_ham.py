"""Pins of the oracle's cell blocks H0, H+, H- (paper Sec. 2, Eqs. 2-4).

The decisive check builds the Hamiltonian of a three-cell supercell that is
simply periodic along z, by plain loops over grid points written here
independently of the oracle, and reads the cell blocks off it: the block that
couples cell 0 to itself is H0, to cell 1 is H+, to cell 2 (= cell -1) is H-.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ham
from oracle.fd import fd_weights_exact
from oracle.qep import P_dense, dispersion_1d


def _supercell(sys, ncell=3):
    nx, ny, nz, h = sys.nx, sys.ny, sys.nz, sys.h
    p = sys.fd_order // 2
    c = [float(v) for v in fd_weights_exact(p)]
    NZ = ncell * nz
    n = nx * ny * NZ
    H = np.zeros((n, n))

    def lin(ix, iy, iz):
        return (ix % nx) + nx * ((iy % ny) + ny * (iz % NZ))
    for iz in range(NZ):
        for iy in range(ny):
            for ix in range(nx):
                i = lin(ix, iy, iz)
                H[i, i] += sys.v_loc[ix + nx * (iy + ny * (iz % nz))]
                for m in range(-p, p + 1):
                    for j in (lin(ix + m, iy, iz), lin(ix, iy + m, iz), lin(ix, iy, iz + m)):
                        H[i, j] += -0.5 * c[m + p] / (h * h)
    pr = sys.proj
    if pr is not None:
        for a in range(pr.n_atoms):
            lo, hi = pr.ball_off[a], pr.ball_off[a + 1]
            for cell in range(ncell):           # periodic images of the atom
                for k in range(pr.n_proj):
                    u = np.zeros(n)
                    for e in range(lo, hi):
                        r = int(pr.ball_idx[e])
                        ix, iy, iz = r % nx, (r // nx) % ny, r // (nx * ny)
                        u[lin(ix, iy, iz + nz * (int(pr.ball_w[e]) + cell))] += pr.ball_val[e, k]
                    H += pr.coeff[a, k] * np.outer(u, u)
    return H


@pytest.mark.parametrize("fd_order,with_proj", [(4, False), (4, True), (8, True)])
def test_blocks_equal_supercell(fd_order, with_proj):
    sys = W.tiny(with_proj=with_proj, fd_order=fd_order)
    Hs = _supercell(sys)
    n = sys.n
    h0, hp, hm = ham.build(sys).blocks_dense()
    np.testing.assert_allclose(h0, Hs[:n, :n], atol=1e-12)
    np.testing.assert_allclose(hp, Hs[:n, n:2 * n], atol=1e-12)
    np.testing.assert_allclose(hm, Hs[:n, 2 * n:], atol=1e-12)


def test_structure_invariants():
    sys = W.tiny(with_proj=True, fd_order=8)
    h0, hp, hm = ham.build(sys).blocks_dense()
    np.testing.assert_allclose(h0, h0.T, atol=1e-13)
    np.testing.assert_allclose(hm, hp.T, atol=0)
    for th in (0.3, 1.7, -2.2):
        P = P_dense(h0, hp, hm, 0.1, np.exp(1j * th))
        np.testing.assert_allclose(P, P.conj().T, atol=1e-12)   # Hermitian on |z| = 1
    z = 1.7 * np.exp(0.4j)
    np.testing.assert_allclose(P_dense(h0, hp, hm, 0.1, z).conj().T,
                               P_dense(h0, hp, hm, 0.1, 1 / np.conj(z)), atol=1e-12)
    np.testing.assert_allclose(P_dense(h0, hp, hm, 0.1, z).T,
                               P_dense(h0, hp, hm, 0.1, 1 / z), atol=1e-12)


def test_free_operator_rank_of_hplus():
    # without projectors H+ only holds the z wrap: rank nx*ny*p
    sys = W.free_system(4, 3, 6, 0.5, 8)
    _, hp, _ = ham.build(sys).blocks_dense()
    assert np.linalg.matrix_rank(hp) == 4 * 3 * 4


def test_plane_wave_eigenvalue():
    # a Bloch plane wave is an eigenvector of the free P(z) with the FD dispersion
    nx, ny, nz, h, p = 6, 5, 7, 0.35, 2
    sys = W.free_system(nx, ny, nz, h, 2 * p)
    H = ham.build(sys)
    mu = 1.3 * np.exp(0.7j)
    lam = mu ** nz
    kx, ky = 2, 3
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    psi = (np.exp(2j * np.pi * (kx * ix / nx + ky * iy / ny)) * mu ** iz).transpose(2, 1, 0).reshape(-1)
    from oracle.fd import fd_weights
    c = fd_weights(p)
    ez = -0.5 * sum(c[m + p] * mu ** m for m in range(-p, p + 1)) / h ** 2
    eps = (dispersion_1d(p, h, np.array([2 * np.pi * kx / nx]))[0]
           + dispersion_1d(p, h, np.array([2 * np.pi * ky / ny]))[0] + ez)
    E = 0.25
    y = H.apply(lam, psi, E)
    np.testing.assert_allclose(y, (eps - E) * psi, rtol=0, atol=1e-10 * np.abs(psi).max() * abs(eps))


def test_sparse_apply_matches_dense():
    sys = W.tiny(with_proj=True, fd_order=8)
    H = ham.build(sys)
    h0, hp, hm = H.blocks_dense()
    rng = np.random.default_rng(5)
    x = rng.standard_normal((sys.n, 3)) + 1j * rng.standard_normal((sys.n, 3))
    for z in (2.0 * np.exp(0.3j), 0.5 * np.exp(-1.1j), np.exp(2.0j)):
        np.testing.assert_allclose(H.apply(z, x, 0.3), P_dense(h0, hp, hm, 0.3, z) @ x, atol=1e-11)
