#!/usr/bin/env python3
"""Throughput of the fully implicit Runge-Kutta stage solve on one MI355X.

Workload (the headline configuration): variable-coefficient diffusion on the
unit square, Q1 on a uniform 1024 x 1024 grid (1,046,529 interior DoFs),
per-element kappa = exp(g) with g a seeded Gaussian random field (std 1,
correlation length 0.1), Radau IIA s = 3, dt = 1e-3, u0 = 16 seeded sine modes;
FGMRES(30) to 1e-10 relative residual, block lower-triangular stage
preconditioner, one geometric-multigrid V-cycle (Chebyshev degree 2) per
diagonal block. A bench "step" is one time step (stage right-hand side, the
FGMRES stage solve with its preconditioner, the update). The timed value uses
the mixed form (FP32 multigrid inside FP64 FGMRES); the FP64 form is measured in
the same run and reported beside it.

Metric: DoF-stage-steps/s = n * s * steps / time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DoF-stage-steps/s at 1e-8 rel. error, RadauIIA s=3, 1024² Q1; mixed vs FP64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--precision", choices=["f32", "bf16", "f64"], default="f32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond", choices=["gs", "jacobi"], default="gs")
    ap.add_argument("--orth", choices=["cgs2", "selective"], default="cgs2")
    ap.add_argument("--guess", choices=["zero", "prev"], default="zero")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--coarse-n", type=int, default=32)
    return ap.parse_args()


def solver_options(P, args):
    return dict(precond={"gs": P.PC_GS_LOWER, "jacobi": P.PC_JACOBI}[args.precond],
                orth={"cgs2": P.ORTH_CGS2, "selective": P.ORTH_CGS_SELECTIVE}[args.orth],
                initial_guess={"zero": P.GUESS_ZERO, "prev": P.GUESS_PREV}[args.guess],
                restart=args.restart, mg_coarse_n=args.coarse_n, rtol=1e-10)


def timed_run(P, torch, prob, tab, dt, u0_dev, steps, warmup, prec, opts):
    stp = P.Stepper(prob, tab, dt, mg_precision=prec, **opts)
    if warmup > 0:
        uw = u0_dev.clone()
        stp.advance(uw, warmup)
    u = u0_dev.clone()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    _, stats = stp.advance(u, steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    return stp, u, ms, stats


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (multi-GPU sharding is a "
                                   "design note, not built)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2403_08084_amd as P
    import synth

    N = args.N
    n = (N - 1) ** 2
    s = 3
    dt = 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    prob = P.Problem(N, torch.as_tensor(kap).cuda())
    tab = P.tableaux.radau_iia(3)
    u0d = torch.as_tensor(u0).cuda()
    prec = {"f32": P.F32, "bf16": P.BF16, "f64": P.F64}[args.precision]
    opts = solver_options(P, args)
    stp, u, ms, stats = timed_run(P, torch, prob, tab, dt, u0d, args.steps, args.warmup, prec, opts)
    value = n * s * args.steps / (ms / 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF-stage-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f64+f32", "bf16": "f64+bf16", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"heat/diffusion Q1 {N}x{N}, GRF kappa (seed 1), RadauIIA(3), dt=1e-3, "
                               f"FGMRES(30) rtol 1e-10, P_L + 1 GMG V-cycle Cheb(2), MG {args.precision}",
                   "N": N, "dofs": n, "stages": s, "global_batch": 1, "seq_len": 0, "parallelism": "none"},
        "fgmres_its_per_step": stats["fgmres_its_total"] / max(1, args.steps),
        "solver": {"precond": args.precond, "orth": args.orth, "guess": args.guess, "restart": args.restart,
                   "coarse_n": args.coarse_n},
    }
    if not args.no_fp64 and prec != P.F64:
        _, u64, ms64, st64 = timed_run(P, torch, prob, tab, dt, u0d, args.steps, args.warmup, P.F64, opts)
        out["fp64"] = {"value": n * s * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps,
                       "fgmres_its_per_step": st64["fgmres_its_total"] / max(1, args.steps)}
        out["mixed_over_fp64"] = value / out["fp64"]["value"]
        uh, u64h = u.cpu().numpy(), u64.cpu().numpy()
        out["rel_diff_mixed_vs_fp64"] = float(np.linalg.norm(uh - u64h) / np.linalg.norm(u64h))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
