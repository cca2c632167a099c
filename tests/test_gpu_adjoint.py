"""Adjoint d lambda / d V_loc (left vectors from the pair partner 1/conj(lambda)).

Checked against the oracle's dense gradient (QZ left/right eigenvectors), through
the chain rule to Gaussian amplitudes with torch autograd, and against
Richardson-extrapolated central differences of the device solve.
Bar: relative error <= 1e-7 against the dense gradient (eigenvectors are accurate
to ~1e-10, the gradient is a product of two of them over a denominator of order 1).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, ham, qep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny_setup():
    sysw = W.tiny(with_proj=True, fd_order=8)
    H = ham.build(sysw)
    h0, hp, hm = H.blocks_dense()
    ref = qep.solve_dense(h0, hp, hm, 4.0, 0.5)
    g = np.stack([W.gaussian_basis(sysw, a) for a in range(len(sysw.amps))])
    return sysw, (h0, hp, hm), ref, g


def _solve(sysw, cuda, E=4.0, L=8, real_v=False, precision=0):
    import torch
    import paper_1709_09347_amd as cbs
    s = cbs.System.from_workload(sysw)
    V = torch.from_numpy(W.make_rhs(sysw.n, L, 3, real=real_v)).to(cuda)
    prm = cbs.default_params(n_rhs=L, n_mom=8, precision=precision)
    lam, vecs, res, info, rc = s.solve(E, V, prm)
    assert rc == 0 and info.nodes_solved == (16 if real_v else 32)
    return s, V, prm, lam


@pytest.mark.parametrize("real_v,precision", [(False, 0), (True, 0), (True, 1)])
def test_grad_vloc_matches_dense(cuda, tiny_setup, real_v, precision):
    # real V: half the nodes solved (the mirrored ones by conjugation); the left vectors are
    # still the partners' eigenvectors from the extraction, so the gradient is the same; in
    # mixed precision (the bench configuration) the eigenvectors come from the refined solves
    sysw, (h0, hp, hm), ref, g = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda, real_v=real_v, precision=precision)
    sel = list(range(len(lam)))
    G = s.grad_vloc(sel).cpu().numpy()
    for k, l in enumerate(lam):
        j = int(np.argmin(np.abs(ref.lam - l)))
        want = adjoint.dlambda_dv(hp, hm, ref.lam[j], ref.x[:, j], ref.y[:, j])
        err = np.abs(G[k] - want).max() / np.abs(want).max()
        assert err <= 1e-7, (l, err)


def test_vjp_and_autograd_chain_to_amplitudes(cuda, tiny_setup):
    import torch
    import paper_1709_09347_amd as cbs
    sysw, (h0, hp, hm), ref, g = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda)
    amps = torch.tensor(sysw.amps, dtype=torch.float64, requires_grad=True)
    gt = torch.from_numpy(g)
    out = cbs.cbs_eig(amps @ gt, s, 4.0, V, prm)
    w = torch.linspace(0.5, 1.5, len(out), dtype=torch.float64)
    loss = (w * (out.real ** 2 + 2 * out.imag)).sum()
    loss.backward()
    # dense reference: dL/dA = sum_k Re(dL/dlam_k-conj-Wirtinger * conj(dlam/dA)) * 2 ...
    want = np.zeros(len(amps))
    for k, l in enumerate(out.detach().numpy()):
        j = int(np.argmin(np.abs(ref.lam - l)))
        dl = adjoint.dlambda_damp(g, adjoint.dlambda_dv(hp, hm, ref.lam[j], ref.x[:, j], ref.y[:, j]))
        # L = w (x^2 + 2 y): dL/dA = w (2 x dx/dA + 2 dy/dA)
        want += float(w[k]) * (2 * l.real * dl.real + 2 * dl.imag)
    np.testing.assert_allclose(amps.grad.numpy(), want, rtol=1e-6, atol=1e-9)


def test_autograd_vs_richardson_differences(cuda, tiny_setup):
    # the autograd gradient of L = sum_k w_k (Re lam_k + 2 Im lam_k) with respect to the
    # Gaussian amplitudes against Richardson-extrapolated central differences of the
    # device solve itself (plain central differences carry an error of order eps^2 times
    # the third derivative, which is large for eigenvalues near a branch point; Richardson
    # removes it).  Solves refined to 1e-13 keep the eigenvalue noise near 5e-12.
    import torch
    import paper_1709_09347_amd as cbs
    sysw, _, _, g = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda)
    prm.tol = 1e-13
    gt = torch.from_numpy(g)
    amps0 = torch.tensor(sysw.amps, dtype=torch.float64)
    w = torch.linspace(0.5, 1.5, len(lam), dtype=torch.float64)

    def loss(a):
        out = cbs.cbs_eig(a @ gt, s, 4.0, V, prm)
        assert len(out) == len(w)
        return (w * (out.real + 2 * out.imag)).sum()

    amps = amps0.clone().requires_grad_(True)
    loss(amps).backward()
    got = amps.grad.numpy()
    want = np.zeros(len(amps0))
    for j in range(len(amps0)):
        def d(h):
            e = torch.zeros_like(amps0)
            e[j] = h
            with torch.no_grad():
                return (float(loss(amps0 + e)) - float(loss(amps0 - e))) / (2 * h)
        want[j] = (4 * d(1e-5) - d(2e-5)) / 3
    err = np.abs(got - want).max() / np.abs(want).max()
    print("autograd", got, "richardson", want, "rel err", err)
    assert err <= 1e-5


def test_grad_rejects_bad_selection(cuda, tiny_setup):
    import paper_1709_09347_amd as cbs
    sysw, _, _, _ = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda)
    with pytest.raises(cbs.CbsError):
        s.grad_vloc([len(lam) + 3])


def test_gradcheck_amplitudes(cuda, tiny_setup):
    # torch.autograd.gradcheck of lambda(A) = cbs_eig(sum_a A_a g_a) on the tiny cell: the
    # adjoint's vector-Jacobian products (real and imaginary part of every eigenvalue) against
    # gradcheck's own central differences of the device solve.  gradcheck runs all its
    # forwards before the backward, so backward cannot rely on the system's last solve.
    # Solves refined to 1e-13 keep the eigenvalue noise (~5e-12) far below eps * atol.
    import torch
    import paper_1709_09347_amd as cbs
    sysw, _, _, g = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda)
    prm.tol = 1e-13
    gt = torch.from_numpy(g)

    def f(a):
        return cbs.cbs_eig(a @ gt, s, 4.0, V, prm)

    amps = torch.tensor(sysw.amps, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(f, (amps,), eps=1e-6, atol=1e-5, rtol=1e-4)


def test_backward_after_another_forward_on_the_same_system(cuda, tiny_setup):
    # two cbs_eig calls on one system with different potentials, then the backward of the
    # first: it must be the gradient at the first potential (the same as a lone
    # forward + backward there), not at the eigenpairs of the later solve
    import torch
    import paper_1709_09347_amd as cbs
    sysw, _, _, g = tiny_setup
    s, V, prm, lam = _solve(sysw, cuda)
    gt = torch.from_numpy(g)
    a0 = torch.tensor(sysw.amps, dtype=torch.float64)

    def grad_of(a, interleave):
        a = a.clone().requires_grad_(True)
        out = cbs.cbs_eig(a @ gt, s, 4.0, V, prm)
        if interleave:
            cbs.cbs_eig((1.05 * a0) @ gt, s, 4.0, V, prm)   # another forward in between
        w = torch.linspace(0.5, 1.5, len(out), dtype=torch.float64)
        (w * (out.real + 2 * out.imag)).sum().backward()
        return a.grad.numpy().copy()

    alone = grad_of(a0, False)
    inter = grad_of(a0, True)
    np.testing.assert_allclose(inter, alone, rtol=1e-9, atol=1e-12)
