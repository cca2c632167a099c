"""The chunked projector bra (the direction of a group of runs staged in LDS chunk by chunk,
every ball entry of the chunk contracted from there) against dense LU, the oracle's BiCG
and the per-atom bra (paper Sec. 4: separable nonlocal projectors; Sec. 3.2: BiCG).

The bra sits inside the operator, so the tests pick it with CBS_BRA_TILE (read when a
system is first tuned: 0 = per atom, 4 / 8 = chunked with that many runs per
workgroup, on chunks of 512 points or, with ":256", of 256; a third field for the
table loads: 0 per lane, 1 shared by the four lanes of a quad) and check what BiCG and the
solve return.  Bars: on the 5x5x8 cell every
solution's residual, recomputed by the oracle, <= 1e-10 and the solution within 1e-8 of LU;
at 48x48x32 (full size) BiCG capped at 20 iterations against the oracle's BiCG after the
same 20 steps on its sparse operator, iterates to 1e-10 relative (the same recurrences:
only the order in which the bra adds separates them); the two table-load modes, which add
in the same order, bit for bit against each other; the full mixed-precision solve with the
chunked bra against the per-atom bra, eigenvalues to 1e-9 relative.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ham, qep, ss

pytestmark = pytest.mark.gpu


def _system(monkeypatch, sysw, rg):
    import paper_1709_09347_amd as cbs
    monkeypatch.setenv("CBS_BRA_TILE", str(rg))
    monkeypatch.setenv("CBS_AUTOTUNE", "0")
    return cbs.System.from_workload(sysw)


@pytest.mark.parametrize("rg", ["4", "8", "4:256", "8:256", "4:512:1", "4:256:1", "8:512:1", "8:256:1"])
@pytest.mark.parametrize("precision", [0, 1])
def test_chunked_bra_tiny_vs_lu(cuda, monkeypatch, rg, precision):
    import torch
    import paper_1709_09347_amd as cbs
    sysw = W.tiny(with_proj=True, fd_order=8)
    h0, hp, hm = ham.build(sysw).blocks_dense()
    E = 0.7
    z1, _, z2, _ = ss.quadrature(0.5, 32)
    V = W.make_rhs(sysw.n, 4, 11)
    s = _system(monkeypatch, sysw, rg)
    Y, Yt, iters, relres, info, rc = s.bicg(E, z1, torch.from_numpy(V).to(cuda),
                                            cbs.default_params(precision=precision))
    assert rc == 0 and relres.max() <= 1e-10
    Y, Yt = Y.cpu().numpy(), Yt.cpu().numpy()
    for j in range(len(z1)):
        A1 = qep.P_dense(h0, hp, hm, E, z1[j])
        A2 = qep.P_dense(h0, hp, hm, E, z2[j])
        for l in range(V.shape[0]):
            nv = np.linalg.norm(V[l])
            assert np.linalg.norm(V[l] - A1 @ Y[j, l]) <= 1e-10 * nv
            assert np.linalg.norm(V[l] - A2 @ Yt[j, l]) <= 1e-10 * nv
            ref = np.linalg.solve(A1, V[l])
            assert np.linalg.norm(Y[j, l] - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("rg", ["4", "8", "4:256", "8:256", "4:512:1", "8:512:1"])
def test_chunked_bra_cfg2_iterates_match_the_oracle(cuda, monkeypatch, rg):
    import torch
    import paper_1709_09347_amd as cbs
    w = W.config(2)
    sysw = w.systems[0]
    E = w.solve.energies[0]
    H = ham.build(sysw)
    z1, _, z2, _ = ss.quadrature(0.5, 32)
    j, L = 5, 2
    V = W.make_rhs(sysw.n, L, 11)
    s = _system(monkeypatch, sysw, rg)
    Y, Yt, iters, relres, info, rc = s.bicg(E, z1[[j]], torch.from_numpy(V).to(cuda),
                                            cbs.default_params(precision=0, max_iter=20))
    assert rc == cbs.CBS_ENOCONV and iters.min() == iters.max() == 20
    Y, Yt = Y.cpu().numpy(), Yt.cpu().numpy()
    for l in range(L):
        x, xt, _, rr, rrt = ss.bicg(lambda u: H.apply(z1[j], u, E), lambda u: H.apply(z2[j], u, E),
                                    V[l], V[l], fixed_iters=20)
        assert np.linalg.norm(Y[0, l] - x) <= 1e-10 * np.linalg.norm(x)
        assert np.linalg.norm(Yt[0, l] - xt) <= 1e-10 * np.linalg.norm(xt)
        assert abs(relres[0, l, 0] - rr) <= 1e-8 * rr and abs(relres[0, l, 1] - rrt) <= 1e-8 * rrt


@pytest.mark.parametrize("tile", ["4:512", "8:512", "4:256"])
@pytest.mark.parametrize("precision", [0, 1])
def test_chunked_bra_table_load_modes_agree_bit_for_bit(cuda, monkeypatch, tile, precision):
    """Three right-hand sides at one node: 3 runs, so the last quad of every group of 4 (or 8)
    runs holds empty run slots, which walk their piece with the others.  In mixed precision
    the runs narrow to complex64 after a few iterations (inner_tol 0.5), so the complex64
    bra is compared too."""
    import torch
    import paper_1709_09347_amd as cbs
    w = W.config(2)
    sysw = w.systems[0]
    E = w.solve.energies[0]
    z1, _, _, _ = ss.quadrature(0.5, 32)
    V = torch.from_numpy(W.make_rhs(sysw.n, 3, 11)).to(cuda)
    prm = cbs.default_params(precision=precision, max_iter=30)
    prm.inner_tol = 0.5
    out = {}
    modes = ("0", "1")
    for mode in modes:
        s = _system(monkeypatch, sysw, f"{tile}:{mode}")
        Y, Yt, iters, relres, info, rc = s.bicg(E, z1[[5]], V, prm)
        assert rc == cbs.CBS_ENOCONV and iters.min() == 30
        out[mode] = (Y.cpu().numpy(), Yt.cpu().numpy(), relres.copy())
        del s
    for mode in modes[1:]:
        for a, b in zip(out[modes[0]], out[mode]):
            assert np.array_equal(a, b), f"table-load mode {mode} differs from mode {modes[0]}"


def test_chunked_bra_cfg2_mixed_solve_matches_the_per_atom_bra(cuda, monkeypatch):
    import torch
    import paper_1709_09347_amd as cbs
    w = W.config(2)
    sysw = w.systems[0]
    E = w.solve.energies[0]
    V = torch.from_numpy(W.make_rhs(sysw.n, 16, w.seed_rhs, real=True)).to(cuda)
    prm = cbs.default_params(n_rhs=16, n_mom=8, precision=cbs.CBS_MIXED)
    out = {}
    for rg in ("0", "8"):
        s = _system(monkeypatch, sysw, rg)
        lam, _, res, info, rc = s.solve(E, V, prm, want_vectors=False)
        assert rc == 0 and len(lam) >= 2 and res.max() <= 1e-8
        out[rg] = (np.asarray(lam), info.iters_mean)
        print(f"bra {rg}: {len(lam)} eigenvalues, mean BiCG iterations {info.iters_mean:.1f}")
    a, b = out["0"][0], out["8"][0]
    assert len(a) == len(b) and qep.match_sets(a, b) <= 1e-9
