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
STENCIL_TRAFFIC_RATIO = 1.0329


def cpu_baseline(sysw, E, V, iters_per_run, n_runs, budget_s=12.0):
    """The oracle's BiCG (scipy.sparse operator) on one run, time-bounded, extrapolated."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ham, ss
    H = ham.build(sysw)
    z1, _, _, _ = ss.quadrature(0.5, 32)
    z = z1[0]
    v = V[0]
    done, t_used = 0, 0.0
    with threadpool_limits(limits=1):
        while t_used < budget_s:
            t0 = time.perf_counter()
            ss.bicg(lambda u: H.apply(z, u, E), lambda u: H.apply(1 / np.conj(z), u, E), v, v,
                    fixed_iters=10)
            t_used += time.perf_counter() - t0
            done += 10
    per_iter = t_used / done
    return {
        "value": per_iter * iters_per_run * n_runs,
        "unit": "s/energy",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{done} BiCG iterations (primal+dual) of one run on the oracle's scipy.sparse "
                   f"operator at this workload ({t_used:.1f} s, 1 thread), extrapolated to {n_runs} runs "
                   f"x {iters_per_run:.0f} iterations (the GPU FP64 solve's mean; the oracle solves "
                   f"every node); moments and extraction not included"),
    }


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", choices=("both", "fp64", "mixed", "mixed_complex_rhs", "mixed_half_stop"),
                    default="both",
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
    if args.legs != "both":
        names = (args.legs,)
    elif args.iters_cap > 0:
        names = ("fp64", "mixed")
    else:
        names = ("fp64", "mixed", "mixed_complex_rhs", "mixed_half_stop")
    # mixed_half_stop: the load-balancing stop of Sec. 3.3 (all solves end once more than
    # half of the nodes converged), reported beside the headline, which solves every run
    legs = [(n, p, v, h) for n, p, v, h in (("fp64", cbs.CBS_FP64, V, 0), ("mixed", cbs.CBS_MIXED, V, 0),
                                            ("mixed_complex_rhs", cbs.CBS_MIXED, Vz, 0),
                                            ("mixed_half_stop", cbs.CBS_MIXED, V, 1)) if n in names]
    for name, prec, Vl, half in legs:
        prm = cbs.default_params(n_rhs=L, n_mom=M, precision=prec, half_stop=half)
        if args.iters_cap > 0:
            prm.max_iter = args.iters_cap
        for _ in range(args.warmup):
            s.solve(E, Vl, prm, want_vectors=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lam, _, res, info, rc = s.solve(E, Vl, prm, want_vectors=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        runs[name] = dict(t=dt, lam=lam, res=res, info=info, rc=rc)
        print(f"# {name}: {dt:.3f} s/energy, {len(lam)} eigenvalues, rank {info.rank}, nodes solved "
              f"{info.nodes_solved}, BiCG iters max {info.iters_max} mean {info.iters_mean:.1f}, max solve "
              f"residual {info.max_solve_resid:.2e}, max eigen residual {info.max_eig_resid:.2e}, rc {rc}",
              file=sys.stderr, flush=True)

    ty64, ty32, tune_log = s.tiling()
    tiling = {"tile_y_c128": ty64, "tile_y_c64": ty32}
    print(f"# stencil tiles: {tiling}; autotuner: {tune_log}", file=sys.stderr, flush=True)
    if args.legs != "both" or args.iters_cap > 0:
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

    mixed, fp64 = runs["mixed"], runs["fp64"]
    dl = qep.match_sets(mixed["lam"], fp64["lam"]) if len(mixed["lam"]) == len(fp64["lam"]) else None
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
        "lambda_rel_diff_mixed_vs_fp64": dl,
        "max_eig_resid": float(max(mixed["info"].max_eig_resid, fp64["info"].max_eig_resid)),
        "bicg_iters_mean": {"fp64": fp64["info"].iters_mean, "mixed": mixed["info"].iters_mean},
        "stencil_tiles": tiling,
        "roofline": roof["fp64"],
        "roofline_complex64_stencil": roof["mixed"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysw, E, Vh, fp64["info"].iters_mean, 32 * L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
