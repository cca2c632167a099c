#!/usr/bin/env python3
"""Time per energy of the Sakurai-Sugiura complex-band-structure solve on one MI355X.

Workload: the 48x48x32 cell (h = 0.3 bohr, 8th-order finite differences) with 96
pseudo-atoms on a cylinder of radius 6 bohr (Gaussian local potential plus four
Gaussian-supported projectors each), E = 0.2 Ha, annulus 0.5 < |lambda| < 2,
N_q = 32 nodes per circle, L = 16 real random right-hand sides, M = 8 moments, every
linear solve to a 1e-10 relative residual.  Inputs are seeded and synthetic and
resident in device memory before the timed region.

One step = one complete solve at one energy (BiCG with duals at the nodes, moments,
Hankel SVD, Rayleigh-Ritz extraction, residuals).  The blocks are real and so is V, so
the solutions at the mirrored nodes conj z_j are the conjugates of those at z_j: 16 of
the 32 nodes per circle are solved (256 runs of a system and its dual) and the moments
sum the mirrored pairs.  The mixed-precision path (complex128 BiCG until a run's
residual is below 1e-6, then complex64 vectors and FP32 operator applications with
complex128 residual replacement) is the reported value; the complex128 path is timed
beside it on the same inputs, and the mixed path with complex random V (every node
solved, 512 runs) is timed after them.

The JSON line also carries the roofline of the dominant kernel (the BiCG stencil,
timed per launch with HIP events on the stream it runs on in a diagnostic solve
after the timed region) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time per energy to 1e-10 residual (mixed vs FP64 GPU); stencil HBM GB/s"
# HBM traffic of the complex128 BiCG stencil relative to its algorithmic bytes, from rocprofv3
# FETCH_SIZE and WRITE_SIZE on full-batch dispatches of this workload, each scaled by what the
# counter reads for a plain 1 GiB device copy (bench.py --copy-calibration); the commands and
# raw figures are in profiles/stencil_fp64_48x48x32_counters.md.  None once the kernel changes.
STENCIL_TRAFFIC_RATIO = 1.1093
# solve tolerance of the eigenpair-residual leg: the Rayleigh-Ritz pairs carry 10-15x the
# solve residual at this workload (1.2e-10 from solves to 1e-11), so 5e-12 keeps them
# below 1e-10
EIG_GATE_TOL = 5e-12


def _oracle_bicg_worker(args):
    """One oracle BiCG run (primal + dual) for a fixed number of iterations, in its own
    process with one BLAS thread; returns (iterations, seconds)."""
    cfg, node, col, iters, E = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import ham, ss
    w = W.config(cfg)
    sysw = w.systems[0]
    H = ham.build(sysw)
    z1, _, _, _ = ss.quadrature(0.5, 32)
    v = W.make_rhs(sysw.n, w.solve.n_rhs, w.seed_rhs, real=True)[col]
    z = z1[node]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ss.bicg(lambda u: H.apply(z, u, E), lambda u: H.apply(1 / np.conj(z), u, E), v, v, fixed_iters=iters)
        return iters, time.perf_counter() - t0


def cpu_baseline(sysw, E, iters_per_run, n_runs, n_nodes, L, M, budget_s=10.0):
    """The oracle on the host cores: its BiCG (scipy.sparse operator) on one run per core in
    parallel processes for a bounded number of iterations, extrapolated to the GPU leg's runs
    and mean iteration count, plus its moments and Hankel SVD extraction timed in full on
    solutions of the workload's shape.  The oracle's Rayleigh-Ritz projection is left out: it
    multiplies by the explicitly assembled nonlocal blocks (about 1.7e9 nonzeros here), which
    alone takes minutes at this size."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ss
    cores = os.cpu_count() or 1
    # a calibration run sizes the sample to the budget
    it0, t0 = _oracle_bicg_worker((2, 0, 0, 10, E))
    per_iter_1 = t0 / it0
    iters = max(10, int(budget_s / per_iter_1))
    jobs = [(2, k % n_nodes, (k // n_nodes) % L, iters, E) for k in range(cores)]
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_bicg_worker, jobs)
    wall = time.perf_counter() - t
    done = sum(r[0] for r in res)
    rate = done / wall                               # run-iterations per second, all cores
    t_solve = n_runs * iters_per_run / rate
    # moments + extraction (oracle code, all BLAS threads) on random solutions of the shape
    rng = np.random.default_rng(7)
    N = sysw.n
    z1, w1, z2, w2 = ss.quadrature(0.5, 2 * n_nodes)
    Y = [(rng.standard_normal((N, L)) + 1j * rng.standard_normal((N, L))) for _ in range(n_nodes)]
    Vc = rng.standard_normal((N, L)).astype(np.complex128)
    with threadpool_limits(limits=cores):
        t = time.perf_counter()
        S = ss.moments(Y, [np.conj(y) for y in Y], z1[:n_nodes], w1[:n_nodes], z2[:n_nodes], w2[:n_nodes], 2 * M)
        mu = [Vc.conj().T @ s for s in S]
        ss.extract(mu, S[:M], M, 1e-10)
        t_ext = time.perf_counter() - t
    return {
        "value": round(t_solve + t_ext, 2),
        "unit": "s/energy",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle BiCG (scipy.sparse operator, primal + dual) on {cores} runs in {cores} parallel "
                   f"processes, {iters} iterations each ({wall:.1f} s wall, {rate:.1f} run-iterations/s), "
                   f"extrapolated to the GPU leg's {n_runs} runs x {iters_per_run:.0f} mean iterations "
                   f"({t_solve:.0f} s); plus the oracle's moments and Hankel SVD extraction timed in full "
                   f"on random solutions of the workload's shape ({t_ext:.1f} s, {cores} BLAS threads); "
                   f"its Rayleigh-Ritz projection (explicit nonlocal blocks) is not included"),
    }


def dense_qz_cfg1():
    """The dense oracle (companion pencil, LAPACK QZ) at the 8x8x12 workload: seconds per energy."""
    import workloads as W
    from oracle import ham, qep
    w = W.config(1)
    sysw = w.systems[0]
    h0, hp, hm = ham.build(sysw).blocks_dense()
    t = time.perf_counter()
    r = qep.solve_dense(h0, hp, hm, w.solve.energies[0], 0.5, left=False)
    return {"s_per_energy": round(time.perf_counter() - t, 3), "n": int(sysw.n), "n_eigs": int(len(r.lam))}


def half_stop_summary(half, full, qep):
    """The half-of-the-nodes stop against the same solve with every run to tol."""
    same = len(half["lam"]) == len(full["lam"])
    return {"s_per_energy": round(half["t"], 4),
            "speedup_vs_every_run_to_tol": round(full["t"] / half["t"], 3),
            "bicg_iters_max": int(half["info"].iters_max),
            "bicg_iters_mean": half["info"].iters_mean,
            "max_solve_resid": half["info"].max_solve_resid,
            "max_eig_resid": half["info"].max_eig_resid,
            "n_eigs": int(len(half["lam"])),
            "lambda_rel_diff_vs_every_run_to_tol": (qep.match_sets(half["lam"], full["lam"]) if same else None)}


LEGS = ("fp64", "mixed", "mixed_complex_rhs", "mixed_half_stop", "mixed_eig_gate", "fp64_block")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cfg4", action="store_true", help="skip the 96x96x32 precision workload")
    ap.add_argument("--legs", choices=("all",) + LEGS, default="all",
                    help="time one leg only (profiling); the default runs every leg, which the JSON "
                         "line needs")
    ap.add_argument("--iters-cap", type=int, default=0,
                    help="cap BiCG at this many iterations (short runs for counter collection; "
                         "no JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (the reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (the path would shard by quadrature node and right-hand side; "
              "runs on several GPUs are not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 5 x 1 GiB (read 1 GiB + write 1 GiB per dispatch)", flush=True)
        return

    import paper_1709_09347_amd as cbs
    import workloads as W
    from oracle import qep

    dev = torch.device("cuda:0")
    w = W.config(2)
    sysw = w.systems[0]
    E = w.solve.energies[0]
    L, M = w.solve.n_rhs, w.solve.n_mom
    Vh = W.make_rhs(sysw.n, L, w.seed_rhs, real=True)
    s = cbs.System.from_workload(sysw)
    V = torch.from_numpy(Vh).to(dev)
    Vz = torch.from_numpy(W.make_rhs(sysw.n, L, w.seed_rhs)).to(dev)   # complex V: every node
    torch.cuda.synchronize()

    runs = {}
    if args.legs != "all":
        names = (args.legs,)
    elif args.iters_cap > 0:
        names = ("fp64", "mixed")
    else:
        names = LEGS
    # mixed_half_stop: the load-balancing stop of Sec. 3.3 (all solves end once more than
    # half of the nodes converged), reported beside the headline, which solves every run;
    # mixed_eig_gate: solves to EIG_GATE_TOL so that every eigenpair residual is below 1e-10;
    # fp64_block: block BiCG over the 16 right-hand sides of each node
    legs = {"fp64": (dict(precision=cbs.CBS_FP64), V), "mixed": (dict(precision=cbs.CBS_MIXED), V),
            "mixed_complex_rhs": (dict(precision=cbs.CBS_MIXED), Vz),
            "mixed_half_stop": (dict(precision=cbs.CBS_MIXED, half_stop=1), V),
            "mixed_eig_gate": (dict(precision=cbs.CBS_MIXED, tol=EIG_GATE_TOL), V),
            "fp64_block": (dict(precision=cbs.CBS_FP64, block=L), V)}
    for name in names:
        kw, Vl = legs[name]
        prm = cbs.default_params(n_rhs=L, n_mom=M, **kw)
        if args.iters_cap > 0:
            prm.max_iter = args.iters_cap
        # the headline pair runs the requested steps; the other legs one warm-up and up to 3 steps
        main_leg = name in ("fp64", "mixed")
        for _ in range(args.warmup if main_leg else min(args.warmup, 1)):
            s.solve(E, Vl, prm, want_vectors=False)
        torch.cuda.synchronize()
        steps = args.steps if main_leg else max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(steps):
            lam, _, res, info, rc = s.solve(E, Vl, prm, want_vectors=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        runs[name] = dict(t=dt, lam=lam, res=res, info=info, rc=rc)
        print(f"# {name}: {dt:.3f} s/energy ({steps} steps), {len(lam)} eigenvalues, rank {info.rank}, nodes solved "
              f"{info.nodes_solved}, BiCG iters max {info.iters_max} mean {info.iters_mean:.1f}, max solve "
              f"residual {info.max_solve_resid:.2e}, max eigen residual {info.max_eig_resid:.2e}, restarts "
              f"{info.restarts}, rc {rc}", file=sys.stderr, flush=True)

    ty64, ty32, tune_log = s.tiling()
    tiling = {"tile_y_c128": ty64, "tile_y_c64": ty32}
    print(f"# stencil tiles: {tiling}; autotuner: {tune_log}", file=sys.stderr, flush=True)
    if args.legs != "all" or args.iters_cap > 0:
        return
    # dominant kernel of both paths: the complex128 BiCG stencil (timed per launch with HIP
    # events in a diagnostic solve of the FP64 leg); the complex64 stencil of the mixed leg
    # is reported beside it
    roof = {}
    for name, prec in (("fp64", cbs.CBS_FP64), ("mixed", cbs.CBS_MIXED)):
        prm = cbs.default_params(n_rhs=L, n_mom=M, precision=prec, profile=1)
        _, _, _, pinfo, _ = s.solve(E, V, prm, want_vectors=False)
        if name == "fp64":
            n_l, ms, by = pinfo.stencil_launches, pinfo.stencil_ms, pinfo.stencil_bytes
            kern, ratio = "k_stencil<double,double,4,true>", STENCIL_TRAFFIC_RATIO
        else:
            n_l, ms, by = pinfo.stencil_lo_launches, pinfo.stencil_lo_ms, pinfo.stencil_lo_bytes
            kern, ratio = "k_stencil<float,float,4,true>", None
        avg_ms = ms / max(n_l, 1)
        avg_bytes = by / max(n_l, 1)
        gbs = avg_bytes / (avg_ms * 1e-3) / 1e9
        roof[name] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "traffic": (round(ratio * avg_bytes) if ratio is not None else None),
                      "kernel": kern, "avg_launch_ms": round(avg_ms, 4),
                      "algorithmic_bytes_per_launch": round(avg_bytes), "launches": int(n_l)}
        print(f"# {kern} ({name} leg): {avg_ms:.3f} ms/launch, {gbs:.0f} GB/s over {n_l} launches",
              file=sys.stderr, flush=True)

    # the precision workload: 96x96x32, 384 atoms with projectors, at -0.2 Ha (two
    # evanescent eigenvalues), mixed against complex128, one solve each after the tiling
    # autotuner has run
    cfg4 = None
    if not args.no_cfg4:
        w4 = W.config(4)
        s4w = w4.systems[0]
        E4 = w4.solve.energies[0]
        s4 = cbs.System.from_workload(s4w)
        V4 = torch.from_numpy(W.make_rhs(s4w.n, L, w4.seed_rhs, real=True)).to(dev)
        s4.solve(E4, V4, cbs.default_params(n_rhs=L, n_mom=M, max_iter=2), want_vectors=False)
        r4 = {}
        for name, prec in (("fp64", cbs.CBS_FP64), ("mixed", cbs.CBS_MIXED)):
            prm = cbs.default_params(n_rhs=L, n_mom=M, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, _, res, info, rc = s4.solve(E4, V4, prm, want_vectors=False)
            torch.cuda.synchronize()
            r4[name] = dict(t=time.perf_counter() - t0, lam=lam, info=info, rc=rc)
            print(f"# cfg4 {name}: {r4[name]['t']:.2f} s/energy, {len(lam)} eigenvalues {lam}, BiCG iters mean "
                  f"{info.iters_mean:.0f} max {info.iters_max}, max solve residual {info.max_solve_resid:.2e}, "
                  f"restarts {info.restarts}, rc {rc}", file=sys.stderr, flush=True)
        same = len(r4["mixed"]["lam"]) == len(r4["fp64"]["lam"])
        cfg4 = {"workload": "96x96x32 h=0.3 fd8, 384 atoms x 4 projectors, E=-0.2 Ha, N_q=32, L=16 real V, M=8, "
                            "BiCG to 1e-10",
                "fp64_s_per_energy": round(r4["fp64"]["t"], 3), "mixed_s_per_energy": round(r4["mixed"]["t"], 3),
                "speedup_mixed_vs_fp64": round(r4["fp64"]["t"] / r4["mixed"]["t"], 3),
                "n_eigs": int(len(r4["mixed"]["lam"])),
                "lambda_rel_diff_mixed_vs_fp64": (qep.match_sets(r4["mixed"]["lam"], r4["fp64"]["lam"])
                                                  if same else None),
                "bicg_iters_mean": {"fp64": r4["fp64"]["info"].iters_mean, "mixed": r4["mixed"]["info"].iters_mean},
                "rc": {"fp64": int(r4["fp64"]["rc"]), "mixed": int(r4["mixed"]["rc"])}}
        s4.close()

    mixed, fp64 = runs["mixed"], runs["fp64"]

    def rel(a, b):
        return qep.match_sets(a["lam"], b["lam"]) if len(a["lam"]) == len(b["lam"]) else None

    gate, blk = runs["mixed_eig_gate"], runs["fp64_block"]
    out = {
        "metric": METRIC,
        "value": round(mixed["t"], 4),
        "unit": "s/energy",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["t"] * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": "48x48x32 h=0.3 fd8, 96 atoms x 4 projectors, E=0.2 Ha, N_q=32, "
                               "L=16 real random V (16 of 32 nodes per circle solved, the mirrored "
                               "ones by conjugation), M=8, BiCG to 1e-10",
                   "global_batch": mixed["info"].nodes_solved * L, "seq_len": sysw.n,
                   "parallelism": "none"},
        "fp64_s_per_energy": round(fp64["t"], 4),
        "speedup_mixed_vs_fp64": round(fp64["t"] / mixed["t"], 3),
        "mixed_complex_rhs_s_per_energy": round(runs["mixed_complex_rhs"]["t"], 4),
        "nodes_solved": {"real_rhs": mixed["info"].nodes_solved,
                         "complex_rhs": runs["mixed_complex_rhs"]["info"].nodes_solved},
        "n_eigs": int(len(mixed["lam"])),
        "half_stop": half_stop_summary(runs["mixed_half_stop"], mixed, qep),
        "eig_gate": {"solve_tol": EIG_GATE_TOL, "s_per_energy": round(gate["t"], 4),
                     "max_eig_resid": gate["info"].max_eig_resid,
                     "bicg_iters_mean": gate["info"].iters_mean,
                     "lambda_rel_diff_vs_tol_1e-10": rel(gate, mixed)},
        "block_bicg": {"block": L, "precision": "c128", "s_per_energy": round(blk["t"], 4),
                       "bicg_iters_mean": blk["info"].iters_mean, "bicg_iters_max": int(blk["info"].iters_max),
                       "max_solve_resid": blk["info"].max_solve_resid, "rc": int(blk["rc"]),
                       "lambda_rel_diff_vs_fp64": rel(blk, fp64)},
        "lambda_rel_diff_mixed_vs_fp64": rel(mixed, fp64),
        "max_eig_resid": float(max(mixed["info"].max_eig_resid, fp64["info"].max_eig_resid)),
        "bicg_iters_mean": {"fp64": fp64["info"].iters_mean, "mixed": mixed["info"].iters_mean},
        "stencil_tiles": tiling,
        "roofline": roof["fp64"],
        "roofline_complex64_stencil": roof["mixed"],
        "cfg4": cfg4,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(sysw, E, fp64["info"].iters_mean, fp64["info"].nodes_solved * L,
                          fp64["info"].nodes_solved, L, M)
        cb["dense_qz_8x8x12"] = dense_qz_cfg1()
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
