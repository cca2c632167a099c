"""Why the large workloads sit at the energies they do: for each energy, BiCG (no
preconditioner, the paper's solver) on a few runs of a workload's cell, capped at a given
number of iterations, and the relative residual it reaches; plus the conventional bands of
H(k) at real k, whose crossings with E count the propagating modes (a lower bound on the
eigenvalues in the annulus).

    python -m workloads.energy_probe --config 5 --energies=-0.6,-0.5,-0.4 --iters 3000

Runs on the GPU through the library (one MI355X); prints one line per energy.
"""
import argparse

import numpy as np


def main():
    import torch
    import paper_1709_09347_amd as cbs
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--energies", default="-0.6,-0.5,-0.4")
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--nodes", default="0,8")
    ap.add_argument("--bands", type=int, default=0)
    ap.add_argument("--nk", type=int, default=9)
    a = ap.parse_args()
    sysw = W.config(a.config).systems[0]
    dev = torch.device("cuda:0")
    s = cbs.System.from_workload(sysw)
    lam_min = 0.5
    nq = 32
    theta = 2 * np.pi * (np.arange(nq) + 0.5) / nq
    z1 = np.exp(1j * theta) / lam_min
    nodes = [int(x) for x in a.nodes.split(",")]
    V = torch.from_numpy(W.make_rhs(sysw.n, 2, 11, real=True)).to(dev)
    cl = sysw.cell_length
    eps = None
    if a.bands > 0:
        ks = np.linspace(0.0, np.pi / cl, a.nk)
        rows = []
        for k in ks:   # one k at a time, so a long band computation reports as it goes
            e, _, _, it, rc = s.bands(np.array([k]), a.bands, tol=1e-9)
            rows.append(e[0])
            print(f"#   k = {k:.5f}: bands {e[0, 0]:.4f} .. {e[0, -1]:.4f} Ha ({it[0]} filter steps, rc {rc})",
                  flush=True)
        eps = np.array(rows)
        print(f"# {sysw.name}: N = {sysw.n}, {a.bands} bands of H(k) at {a.nk} k in [0, pi/a]: lowest "
              f"{eps.min():.4f} Ha, top of the band set {eps[:, -1].min():.4f} Ha; crossings are "
              f"counted only below that top", flush=True)
    for E in (float(x) for x in a.energies.split(",")):
        prm = cbs.default_params(precision=0, max_iter=a.iters)
        Y, Yt, iters, relres, info, rc = s.bicg(E, z1[nodes], V, prm)
        line = (f"E = {E:+.3f} Ha: BiCG after at most {a.iters} iterations: relative residual max "
                f"{relres.max():.2e}, min {relres.min():.2e}, iterations {iters.min()}-{iters.max()} (rc {rc})")
        if eps is not None:
            # propagating modes: band crossings of E over [0, pi/a], both signs of k
            cross = int(np.sum((eps[:-1] - E) * (eps[1:] - E) < 0))
            line += f"; band crossings in [0, pi/a]: {cross} (propagating modes >= {2 * cross})"
        print(line, flush=True)


if __name__ == "__main__":
    main()
