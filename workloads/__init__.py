"""Seeded synthetic inputs for the complex-band-structure (CBS) workloads.

This module produces *input data only*: the real-space grid, the local
potential sampled on it, the separable nonlocal projector tables and the
random right-hand-side block V.  It holds none of the method's arithmetic
(no finite-difference weights, no quadrature, no solves): both the CPU oracle
and the GPU path read these arrays and do their own work on them.

Physical model (Hartree atomic units, bohr):
  * grid nx*ny*nz points of spacing h; x and y periodic (Gamma point),
    z is the transport direction, coupled to neighbouring cells by the Bloch
    factor lambda (paper Sec. 2, Eqs. 2-4);
  * V_loc(r) = sum_a A_a exp(-|r-R_a|^2 / (2 sigma^2)), summed over periodic
    images within 6 sigma; sigma = 0.8 bohr, A_a ~ U[-2, -0.5] Ha;
  * pseudo-atoms with projectors carry four Gaussian-supported projectors
    (s, p_x, p_y, p_z with sigma_p = 1 bohr) truncated at r_c, each scaled so
    that its values u on the ball points have unit 2-norm (u = h^{3/2} p,
    the symmetric grid form of |p><p|); coefficients h_ai ~ U[0.2, 1.0] Ha.
    A ball point at integer grid position (ix, iy, iz) maps to the cell
    point (ix mod nx, iy mod ny, iz mod nz) and carries the cell shift
    w = floor(iz / nz) in {-1, 0, 1};
  * V: entries (a + ib)/sqrt(2), a, b ~ N(0, 1), from numpy's PCG64.

Seeds: atom positions/depths 1000+c, projector coefficients 2000+c,
right-hand sides 3000+c for configuration c.

Layouts:
  * linear point index  n = ix + nx*(iy + ny*iz)
  * V: array [L, N] complex128 (each right-hand side contiguous)
  * projector tables (atom-major, CSR over atoms):
      ball_off [n_atoms+1] int64, ball_idx [nnz] int32, ball_w [nnz] int8,
      ball_val [nnz, n_proj] float64, coeff [n_atoms, n_proj] float64
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GAUSS_SIGMA = 0.8      # bohr, width of the local-potential Gaussians
GAUSS_CUT = 6.0        # images summed within GAUSS_CUT * sigma
PROJ_SIGMA = 1.0       # bohr, width of the projector Gaussians


@dataclasses.dataclass
class Projectors:
    n_atoms: int
    n_proj: int
    ball_off: np.ndarray    # int64 [n_atoms+1]
    ball_idx: np.ndarray    # int32 [nnz]
    ball_w: np.ndarray      # int8  [nnz]
    ball_val: np.ndarray    # float64 [nnz, n_proj]
    coeff: np.ndarray       # float64 [n_atoms, n_proj]

    @property
    def nnz(self) -> int:
        return int(self.ball_off[-1])


@dataclasses.dataclass
class System:
    """One periodic cell: grid, local potential and optional projectors."""
    nx: int
    ny: int
    nz: int
    h: float
    fd_order: int
    v_loc: np.ndarray                    # float64 [N]
    centres: np.ndarray                  # float64 [n_atoms, 3]
    amps: np.ndarray                     # float64 [n_atoms]
    proj: Optional[Projectors] = None
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def p(self) -> int:
        return self.fd_order // 2

    @property
    def cell_length(self) -> float:
        return self.nz * self.h


@dataclasses.dataclass
class SolveConfig:
    """Contour and solver parameters (paper Sec. 3 and Sec. 4.1 values by default)."""
    energies: List[float]
    lambda_min: float = 0.5
    n_q: int = 32
    n_rhs: int = 16
    n_mom: int = 8
    delta: float = 1e-10
    tol: float = 1e-10


@dataclasses.dataclass
class Workload:
    name: str
    systems: List[System]
    solve: SolveConfig
    seed_rhs: int


def _grid_coords(nx, ny, nz, h):
    ix = np.arange(nx) * h
    iy = np.arange(ny) * h
    iz = np.arange(nz) * h
    return ix, iy, iz


def gaussian_potential(nx, ny, nz, h, centres, amps, sigma=GAUSS_SIGMA):
    """V_loc on the grid: sum of Gaussians over periodic images within 6 sigma.

    Evaluated per atom on the local box of grid points around each image, so
    the cost is O(n_atoms * (12 sigma / h)^3) rather than O(n_atoms * N).
    """
    v = np.zeros((nz, ny, nx))
    cut = GAUSS_CUT * sigma
    r = int(math.ceil(cut / h)) + 1
    for (cx, cy, cz), a in zip(np.asarray(centres), np.asarray(amps)):
        # integer grid positions (unwrapped) near the centre
        gx = np.arange(int(math.floor(cx / h)) - r, int(math.floor(cx / h)) + r + 2)
        gy = np.arange(int(math.floor(cy / h)) - r, int(math.floor(cy / h)) + r + 2)
        gz = np.arange(int(math.floor(cz / h)) - r, int(math.floor(cz / h)) + r + 2)
        dx = gx * h - cx
        dy = gy * h - cy
        dz = gz * h - cz
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        val = np.where(d2 <= cut * cut, a * np.exp(-d2 / (2 * sigma * sigma)), 0.0)
        # accumulate onto the periodic cell (np.add.at handles wrap collisions)
        iz_ = np.mod(gz, nz)[:, None, None]
        iy_ = np.mod(gy, ny)[None, :, None]
        ix_ = np.mod(gx, nx)[None, None, :]
        np.add.at(v, (np.broadcast_to(iz_, val.shape), np.broadcast_to(iy_, val.shape),
                      np.broadcast_to(ix_, val.shape)), val)
    return v.reshape(-1)


def gaussian_basis(sys: System, atom: int, sigma=GAUSS_SIGMA) -> np.ndarray:
    """Unit-amplitude Gaussian g_a on the grid (dV_loc/dA_a), periodic images."""
    return gaussian_potential(sys.nx, sys.ny, sys.nz, sys.h, sys.centres[atom:atom + 1],
                              np.ones(1), sigma)


def projector_tables(nx, ny, nz, h, centres, rng_coeff, r_c=3.0, n_proj=4,
                     sigma_p=PROJ_SIGMA) -> Projectors:
    """Ball tables of s, p_x, p_y, p_z Gaussian projectors truncated at r_c."""
    offs = [0]
    idx_l, w_l, val_l = [], [], []
    r = int(math.ceil(r_c / h)) + 1
    for (cx, cy, cz) in np.asarray(centres):
        gx = np.arange(int(math.floor(cx / h)) - r, int(math.floor(cx / h)) + r + 2)
        gy = np.arange(int(math.floor(cy / h)) - r, int(math.floor(cy / h)) + r + 2)
        gz = np.arange(int(math.floor(cz / h)) - r, int(math.floor(cz / h)) + r + 2)
        GZ, GY, GX = np.meshgrid(gz, gy, gx, indexing="ij")
        dx = GX * h - cx
        dy = GY * h - cy
        dz = GZ * h - cz
        d2 = dx * dx + dy * dy + dz * dz
        m = d2 <= r_c * r_c
        dx, dy, dz, d2 = dx[m], dy[m], dz[m], d2[m]
        gxm, gym, gzm = GX[m], GY[m], GZ[m]
        env = np.exp(-d2 / (2 * sigma_p * sigma_p))
        vals = np.stack([env, dx * env, dy * env, dz * env], axis=1)[:, :n_proj]
        vals = vals / np.linalg.norm(vals, axis=0, keepdims=True)
        w = np.floor_divide(gzm, nz)
        lin = np.mod(gxm, nx) + nx * (np.mod(gym, ny) + ny * np.mod(gzm, nz))
        order = np.argsort(lin * 4 + (w + 1), kind="stable")
        idx_l.append(lin[order].astype(np.int32))
        w_l.append(w[order].astype(np.int8))
        val_l.append(vals[order])
        offs.append(offs[-1] + int(m.sum()))
    coeff = rng_coeff.uniform(0.2, 1.0, size=(len(centres), n_proj))
    return Projectors(
        n_atoms=len(centres), n_proj=n_proj,
        ball_off=np.asarray(offs, dtype=np.int64),
        ball_idx=np.concatenate(idx_l) if idx_l else np.zeros(0, np.int32),
        ball_w=np.concatenate(w_l) if w_l else np.zeros(0, np.int8),
        ball_val=np.concatenate(val_l) if val_l else np.zeros((0, n_proj)),
        coeff=coeff)


def make_system(nx, ny, nz, h, fd_order, n_atoms, seed_atoms, seed_coeff=None,
                cylinder_radius=None, with_proj=False, r_c=3.0, name="",
                zero_potential=False) -> System:
    rng = np.random.default_rng(seed_atoms)
    lx, ly, lz = nx * h, ny * h, nz * h
    if cylinder_radius is None:
        centres = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * np.array([lx, ly, lz])
    else:
        phi = rng.uniform(0.0, 2 * math.pi, size=n_atoms)
        zc = rng.uniform(0.0, lz, size=n_atoms)
        centres = np.stack([lx / 2 + cylinder_radius * np.cos(phi),
                            ly / 2 + cylinder_radius * np.sin(phi), zc], axis=1)
    amps = rng.uniform(-2.0, -0.5, size=n_atoms)
    if zero_potential or n_atoms == 0:
        v = np.zeros(nx * ny * nz)
    else:
        v = gaussian_potential(nx, ny, nz, h, centres, amps)
    proj = None
    if with_proj:
        if 2 * r_c >= lz:
            raise ValueError("projector diameter must be below the cell length")
        proj = projector_tables(nx, ny, nz, h, centres, np.random.default_rng(seed_coeff), r_c=r_c)
    return System(nx, ny, nz, h, fd_order, v, centres, amps, proj, name)


def free_system(nx, ny, nz, h, fd_order) -> System:
    """V = 0, no projectors: the free-electron finite-difference crystal."""
    return System(nx, ny, nz, h, fd_order, np.zeros(nx * ny * nz), np.zeros((0, 3)),
                  np.zeros(0), None, f"free_{nx}x{ny}x{nz}")


def make_rhs(n: int, n_rhs: int, seed: int, real: bool = False) -> np.ndarray:
    """Random right-hand sides V as an [L, N] complex128 array: complex Gaussian entries, or
    with real=True real Gaussian entries (stored as complex128 with zero imaginary parts)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n_rhs, n))
    if real:
        return a.astype(np.complex128)
    b = rng.standard_normal((n_rhs, n))
    return (a + 1j * b) / math.sqrt(2.0)


def _atoms_for_area(nx, ny, h):
    # six Gaussians per (8 * 0.4 bohr)^2 of cross-section, as in the smallest cell
    return int(round(6 * (nx * h) * (ny * h) / (3.2 * 3.2)))


def config(c: int) -> Workload:
    """The five synthetic workloads (1-based index c)."""
    if c == 1:
        s = make_system(8, 8, 12, 0.4, 4, 6, 1001, name="cfg1_8x8x12")
        return Workload("cfg1", [s], SolveConfig([0.3], n_rhs=8), 3001)
    if c == 2:
        s = make_system(48, 48, 32, 0.3, 8, 96, 1002, 2002, cylinder_radius=6.0,
                        with_proj=True, name="cfg2_48x48x32")
        return Workload("cfg2", [s], SolveConfig([0.2]), 3002)
    if c == 3:
        systems = []
        for k, n in enumerate((32, 40, 56, 64)):
            systems.append(make_system(n, n, 32, 0.3, 8, _atoms_for_area(n, n, 0.3),
                                       1003 + 10 * k, name=f"cfg3_{n}x{n}x32"))
        return Workload("cfg3", systems, SolveConfig(list(np.linspace(-0.5, 0.5, 16))), 3003)
    if c == 4:
        s = make_system(96, 96, 32, 0.3, 8, 384, 1004, 2004, cylinder_radius=12.0,
                        with_proj=True, name="cfg4_96x96x32")
        # unpreconditioned BiCG converges here at E <= ~0 Ha (~1500 iterations at -0.4 Ha,
        # ~2200 at -0.2, ~4600 at 0, none in 5000 at 0.2 Ha); the annulus holds no eigenvalue
        # at -0.4 Ha, 2 at -0.2 Ha (|lambda| 0.535 and 1.870) and 4 at 0 Ha
        return Workload("cfg4", [s], SolveConfig([-0.2]), 3004)
    if c == 5:
        s = make_system(160, 160, 48, 0.3, 8, 1024, 1005, 2005, cylinder_radius=20.0,
                        with_proj=True, name="cfg5_160x160x48")
        # the lowest-iteration energy probed for BiCG on this cell (residual 4e-6 after 5000
        # iterations at -0.6 Ha, 0.26 at -0.4 Ha)
        return Workload("cfg5", [s], SolveConfig([-0.6]), 3005)
    raise ValueError(f"unknown configuration {c}")


def tiny(with_proj: bool = True, fd_order: int = 4, seed: int = 7) -> System:
    """A 5x5x8 cell (h = 0.45) with three Gaussians, for dense checks in seconds."""
    return make_system(5, 5, 8, 0.45, fd_order, 3, 1100 + seed, 2100 + seed,
                       with_proj=with_proj, r_c=1.5, name=f"tiny_p{fd_order // 2}")
