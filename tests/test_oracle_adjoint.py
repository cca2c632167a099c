"""Pin of the oracle gradient d lambda / d A_a against central differences."""
import numpy as np

import workloads as W
from oracle import adjoint, ham, qep


def _lams(sys, amps, E):
    s2 = W.System(sys.nx, sys.ny, sys.nz, sys.h, sys.fd_order,
                  W.gaussian_potential(sys.nx, sys.ny, sys.nz, sys.h, sys.centres, amps),
                  sys.centres, amps, sys.proj)
    h0, hp, hm = ham.build(s2).blocks_dense()
    return qep.solve_dense(h0, hp, hm, E, 0.5), (h0, hp, hm)


def test_gradient_vs_central_differences():
    sys = W.tiny(with_proj=True, fd_order=8)
    E = 4.0
    base, (h0, hp, hm) = _lams(sys, sys.amps, E)
    g = np.stack([W.gaussian_basis(sys, a) for a in range(len(sys.amps))])
    # the potential really is the sum of the unit Gaussians
    np.testing.assert_allclose(sys.amps @ g, sys.v_loc, atol=1e-12)
    simple = [i for i, l in enumerate(base.lam)
              if np.sum(np.abs(base.lam - l) < 1e-6 * abs(l)) == 1]
    assert simple
    # central differences with steps 2e-5 and 1e-5, combined by Richardson
    # extrapolation (removes the O(eps^2) term, which is large next to the
    # branch points at lambda ~ 1)
    steps = (2e-5, 1e-5)
    pert = {}
    for a in range(len(sys.amps)):
        for eps in steps:
            for sgn in (1, -1):
                amps = sys.amps.copy()
                amps[a] += sgn * eps
                pert[a, eps, sgn] = _lams(sys, amps, E)[0].lam
    for i in simple:
        lam = base.lam[i]
        gv = adjoint.dlambda_dv(hp, hm, lam, base.x[:, i], base.y[:, i])
        ga = adjoint.dlambda_damp(g, gv)
        for a in range(len(sys.amps)):
            d = []
            for eps in steps:
                lp, lm = pert[a, eps, 1], pert[a, eps, -1]
                d.append((lp[np.argmin(np.abs(lp - lam))] - lm[np.argmin(np.abs(lm - lam))]) / (2 * eps))
            rich = (4 * d[1] - d[0]) / 3
            assert abs(rich - ga[a]) <= 1e-7 * max(1.0, abs(ga[a]))


def test_left_vector_is_pair_partner():
    sys = W.tiny(with_proj=True, fd_order=8)
    r, _ = _lams(sys, sys.amps, 4.0)
    for i, l in enumerate(r.lam):
        j = int(np.argmin(np.abs(r.lam - 1 / np.conj(l))))
        if np.sum(np.abs(r.lam - r.lam[j]) < 1e-6) > 1:
            continue
        assert abs(abs(np.vdot(r.y[:, i], r.x[:, j])) - 1) < 1e-8
