"""Cell blocks of the real-space finite-difference Kohn-Sham Hamiltonian.

Paper Sec. 2: in a crystal that is periodic along z only nearest cells
couple (Eq. 2), and the Bloch ansatz psi_{n+l} = lambda^l psi_n (Eq. 3)
turns the Kohn-Sham equation into a quadratic eigenvalue problem (Eq. 4).
With the cell blocks H0 = H_{n,n}, H+ = H_{n,n+1}, H- = H_{n,n-1} = H+^T the
operator used throughout is

    P(z) = (H0 - E) + z H+ + z^{-1} H-.

Contributions (Hartree units):
  * kinetic energy -1/2 Laplacian, central finite differences of half-width p
    on each axis; x and y wrap with phase 1 (Gamma point), a z neighbour that
    leaves the cell through the top lands in H+, through the bottom in H-;
  * local potential V_loc on the diagonal of H0;
  * separable nonlocal projectors: V_nl = sum_{a,i} h_ai |u_ai><u_ai| over all
    periodic images.  Splitting the ball values of atom a by cell shift w
    (u_{ai,w}), the part that couples cell n to cell n+d collects the products
    u_{ai,w} u_{ai,w+d}^T, so H0 gains sum_w h u_w u_w^T and H+ gains
    sum_w h u_w u_{w+1}^T.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .fd import fd_weights


def _periodic_1d(n: int, c: np.ndarray) -> sp.csr_matrix:
    """h^2 * second-derivative matrix on a periodic ring of n points."""
    p = (len(c) - 1) // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        for m in range(-p, p + 1):
            rows.append(i)
            cols.append((i + m) % n)
            vals.append(c[m + p])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def _bloch_1d(n: int, c: np.ndarray):
    """Split the z second-derivative into in-cell, +1-cell and -1-cell parts."""
    p = (len(c) - 1) // 2
    if n < p:
        raise ValueError("cell must hold at least p planes along z")
    d0 = np.zeros((n, n))
    dp = np.zeros((n, n))
    dm = np.zeros((n, n))
    for i in range(n):
        for m in range(-p, p + 1):
            j = i + m
            if j >= n:
                dp[i, j - n] += c[m + p]
            elif j < 0:
                dm[i, j + n] += c[m + p]
            else:
                d0[i, j] += c[m + p]
    return sp.csr_matrix(d0), sp.csr_matrix(dp), sp.csr_matrix(dm)


@dataclasses.dataclass
class Hamiltonian:
    """Sparse cell blocks; local parts as CSR, nonlocal parts as factors."""
    n: int
    loc0: sp.csr_matrix          # -1/2 K_in-cell + diag(V)
    locp: sp.csr_matrix          # -1/2 K_+  (z wrap through the top face)
    # nonlocal factors: U[w] is N x (n_atoms*n_proj) for w = -1, 0, 1
    u: dict
    d: np.ndarray                # coefficients h_ai, flattened like U's columns

    # ---- operator form -------------------------------------------------
    def _nl_blocks(self):
        zero = sp.csr_matrix((self.n, self.n))
        if self.u is None:
            return zero, zero
        D = sp.diags(self.d)
        nl0 = zero.copy()
        nlp = zero.copy()
        for w in (-1, 0, 1):
            nl0 = nl0 + self.u[w] @ D @ self.u[w].T
            if w + 1 in self.u:
                nlp = nlp + self.u[w] @ D @ self.u[w + 1].T
        return nl0, nlp

    def blocks_sparse(self):
        """(H0, H+, H-) as scipy sparse matrices (nonlocal parts made explicit)."""
        nl0, nlp = self._nl_blocks()
        h0 = (self.loc0 + nl0).tocsr()
        hp = (self.locp + nlp).tocsr()
        return h0, hp, hp.T.tocsr()

    def blocks_dense(self):
        h0, hp, hm = self.blocks_sparse()
        return h0.toarray(), hp.toarray(), hm.toarray()

    def apply(self, z: complex, x: np.ndarray, E: float) -> np.ndarray:
        """P(z) x for x of shape [N] or [N, k], without forming V_nl."""
        y = self.loc0 @ x - E * x + z * (self.locp @ x) + (self.locp.T @ x) / z
        if self.u is not None:
            # bra with z^{w}, ket with z^{-w}
            c = sum((z ** w) * (self.u[w].T @ x) for w in (-1, 0, 1))
            c = (self.d[:, None] * c) if c.ndim == 2 else self.d * c
            y = y + sum((z ** (-w)) * (self.u[w] @ c) for w in (-1, 0, 1))
        return y


def build(sys) -> Hamiltonian:
    """Assemble the blocks of one ``workloads.System``."""
    nx, ny, nz, h = sys.nx, sys.ny, sys.nz, sys.h
    c = fd_weights(sys.fd_order // 2)
    dx = _periodic_1d(nx, c)
    dy = _periodic_1d(ny, c)
    dz0, dzp, _dzm = _bloch_1d(nz, c)
    ix, iy, iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    # index n = ix + nx*(iy + ny*iz): z slowest, x fastest
    k_in = (sp.kron(iz, sp.kron(iy, dx)) + sp.kron(iz, sp.kron(dy, ix))
            + sp.kron(dz0, sp.kron(iy, ix))) / (h * h)
    k_p = sp.kron(dzp, sp.kron(iy, ix)) / (h * h)
    loc0 = (-0.5 * k_in + sp.diags(np.asarray(sys.v_loc, dtype=np.float64))).tocsr()
    locp = (-0.5 * k_p).tocsr()
    n = nx * ny * nz
    u = None
    d = np.zeros(0)
    pr = sys.proj
    if pr is not None and pr.n_atoms > 0:
        u = {}
        ncol = pr.n_atoms * pr.n_proj
        atom_of = np.repeat(np.arange(pr.n_atoms), np.diff(pr.ball_off))
        for w in (-1, 0, 1):
            sel = np.nonzero(pr.ball_w == w)[0]
            rows = np.repeat(pr.ball_idx[sel].astype(np.int64), pr.n_proj)
            cols = (atom_of[sel][:, None] * pr.n_proj + np.arange(pr.n_proj)[None, :]).reshape(-1)
            vals = pr.ball_val[sel].reshape(-1)
            u[w] = sp.csr_matrix((vals, (rows, cols)), shape=(n, ncol))
        d = pr.coeff.reshape(-1).astype(np.float64)
    return Hamiltonian(n, loc0, locp, u, d)
