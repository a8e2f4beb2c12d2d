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
the same run and reported beside it, and both are checked against the CPU
oracle's full-size result (tests/golden).

Metric: DoF-stage-steps/s = n * s * steps / time, inputs resident in HBM.
Extra JSON objects: "roofline" (the streaming Gram-Schmidt passes, timed with HIP
events on its launch stream by the library's measurement hook, algorithmic
bytes vs the 8 TB/s HBM3E peak), "cpu_baseline" (the CPU oracle on a bounded
sample of the same workload) and "variants" (the same workload, mixed form,
solved with the Rana-LD preconditioner in the IA form and with the monolithic
multigrid cycle), "copy_ceiling" inside "roofline" (a plain 256 MiB device copy timed
the same way, the bandwidth a streaming kernel can reach in practice) and "adjoint"
(the gradient workload: 512 x 512, Radau IIA(3), 40 steps, 8 snapshots, FP64;
forward and gradient wall times).

Other workloads of the same method: --tableau, --dt, --kappa one, --N, --steps,
--precision, --precond, --splitting, --stage-type.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DoF-stage-steps/s at 1e-8 rel. error, RadauIIA s=3, 1024² Q1; mixed vs FP64"
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "config4_radau3_1024.json")
TRAFFIC = os.path.join(ROOT, "profiles", "gram_schmidt_traffic.txt")
KRYLOV_SRC = os.path.join(ROOT, "paper_2403_08084_amd", "csrc", "k_krylov.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--kappa", choices=["grf", "one"], default="grf",
                    help="per-element diffusivity: exp(GRF seed 1) or 1 everywhere")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient workload")
    ap.add_argument("--precision", choices=["f32", "bf16", "f64"], default="f32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2, help="time steps in the CPU oracle sample")
    ap.add_argument("--precond", choices=["gs", "jacobi", "rana", "gsu", "mmg"], default="gs")
    ap.add_argument("--tableau", choices=["radau3", "radau1", "radau2", "radau4", "gl4", "alexander", "wso433"],
                    default="radau3", help="Butcher tableau (the headline workload is radau3)")
    ap.add_argument("--stage-type", choices=["coupled", "dirk"], default="coupled",
                    help="one coupled stage solve, or stage-by-stage solves for a DIRK tableau")
    ap.add_argument("--splitting", choices=["ai", "ia"], default="ai",
                    help="stage formulation: eq:block_struct_AI (k) or eq:block_struct_IA (w = A k)")
    ap.add_argument("--orth", choices=["cgs2", "selective", "dcgs2"], default="dcgs2")
    ap.add_argument("--guess", choices=["zero", "prev"], default="zero")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--coarse-n", type=int, default=32)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the extra mixed-precision runs of the same workload with the other preconditioners")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy (counter calibration for profiles)")
    return ap.parse_args()


def solver_options(P, args):
    return dict(precond={"gs": P.PC_GS_LOWER, "jacobi": P.PC_JACOBI, "rana": P.PC_RANA_LD, "gsu": P.PC_GS_UPPER,
                          "mmg": P.PC_MONOLITHIC}[args.precond],
                orth={"cgs2": P.ORTH_CGS2, "selective": P.ORTH_CGS_SELECTIVE, "dcgs2": P.ORTH_DCGS2}[args.orth],
                initial_guess={"zero": P.GUESS_ZERO, "prev": P.GUESS_PREV}[args.guess],
                splitting={"ai": P.SPLIT_AI, "ia": P.SPLIT_IA}[args.splitting],
                stage_type={"coupled": P.STAGE_COUPLED, "dirk": P.STAGE_DIRK}[args.stage_type],
                restart=args.restart, mg_coarse_n=args.coarse_n, rtol=1e-10)


def timed_run(P, torch, prob, tab, dt, u0_dev, steps, warmup, prec, opts):
    t0 = time.time()
    stp = P.Stepper(prob, tab, dt, mg_precision=prec, **opts)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
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
    return stp, u, ev0.elapsed_time(ev1), stats, setup_s


def make_tableau(P, name):
    T = P.tableaux
    return {"radau1": lambda: T.radau_iia(1), "radau2": lambda: T.radau_iia(2), "radau3": lambda: T.radau_iia(3),
            "radau4": lambda: T.radau_iia(4), "gl4": lambda: T.gauss_legendre(4), "alexander": T.alexander,
            "wso433": T.wsodirk433}[name]()


def golden_error(u, steps, tableau="radau3", workload_matches=True):
    """Relative L2 error of u against the oracle's full-size result (sketch estimate), or None."""
    import numpy as np

    import synth

    if not workload_matches or not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        g = json.load(f)
    ref = g["steps"].get(str(steps))
    if ref is None or g["n"] != u.size or g.get("tableau") != tableau:
        return None
    G = synth.sketch_vectors(g["n"], g["n_sketch"], g["sketch_seed"])
    idx = np.asarray(g["indices"])
    d = G @ u - np.asarray(ref["sketch"])
    return {"rel_l2_sketch": float(np.sqrt(np.mean(d * d)) / ref["norm2"]),
            "rel_max_samples": float(np.abs(u[idx] - np.asarray(ref["samples"])).max() / ref["norminf"]),
            "rel_norm": float(abs(np.linalg.norm(u) - ref["norm2"]) / ref["norm2"])}


def traffic_bytes_per_launch():
    """Counter-measured HBM bytes per Gram-Schmidt pass (DCGS2 reduction and update) from the committed profile.

    Used only if the summary was taken on the current k_krylov.hip (its sha256 prefix
    is recorded in the summary); otherwise None."""
    if not os.path.exists(TRAFFIC):
        return None
    src = hashlib.sha256(open(KRYLOV_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(TRAFFIC):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != src:
        return None
    try:
        return float(vals["hbm_bytes_per_launch_avg"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(N, steps):
    """The CPU oracle (eigen-decoupled direct tier, one thread) on `steps` steps of the same workload."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, step
    from oracle import tableaux as T
    import synth

    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    tab = T.radau_iia(3)
    with threadpool_limits(1):
        t0 = time.time()
        M, K = fem.assemble(N, kap)
        S = step.DecoupledLU(M, K, tab["A"], 1e-3)
        t1 = time.time()
        u = u0
        for _ in range(steps):
            k = S.solve(step.stage_rhs(K, u, 3))
            u = step.update(u, k, tab["b"], 1e-3)
        t2 = time.time()
    n = (N - 1) ** 2
    return {"value": n * 3 * steps / (t2 - t0), "unit": "DoF-stage-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{N}x{N} RadauIIA(3) workload, assembly + factorisation + {steps} time steps "
                      f"(eigen-decoupled SuperLU, 1 thread)",
            "setup_s": t1 - t0, "solve_s_per_step": (t2 - t1) / max(1, steps)}


def copy_ceiling(torch, mib=256, reps=10):
    """Bandwidth of a plain device-to-device copy (read + write bytes / time), HIP events on the stream."""
    a = torch.ones(mib * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2 * mib * 1024 * 1024 * reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del a, b
    return {"achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "unit": "GB/s",
            "kernel": f"device-to-device copy of {mib} MiB, {reps} times"}


def adjoint_timing(P, torch, synth, N=512, steps=40, nsnap=8, dt=1e-3):
    """Gradient of J = 1/2 |u_N|_M^2 with respect to log kappa (512^2, Radau IIA(3), FP64 multigrid): wall time
    of the forward steps and of the discrete adjoint with binomial checkpointing (graphs captured beforehand)."""
    kap = torch.as_tensor(synth.grf_kappa(N, 1)).cuda()
    u0 = torch.as_tensor(synth.sine_modes_u0(N, 0)[0]).cuda()
    prob = P.Problem(N, kap)
    stp = P.Stepper(prob, P.tableaux.radau_iia(3), dt, mg_precision=P.F64)
    uw = u0.clone()
    stp.advance(uw, 2)
    stp.adjoint(u0, 2, 1, uw)
    u = u0.clone()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    _, fst = stp.advance(u, steps)
    ev[1].record()
    lam = prob.apply_mass(u)
    torch.cuda.synchronize()
    ev[2].record()
    _, _, ast = stp.adjoint(u0, steps, nsnap, lam)
    ev[3].record()
    torch.cuda.synchronize()
    fwd, grad = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    return {"workload": f"gradient of 1/2 |u_N|_M^2 w.r.t. log kappa, Q1 {N}x{N}, kappa=exp(GRF seed 1), Radau IIA(3), "
                        f"dt={dt:g}, {steps} steps, {nsnap} snapshots, P_L, FP64",
            "forward_ms": fwd, "gradient_ms": grad, "gradient_over_forward": grad / fwd,
            "forward_its": fst["fgmres_its_total"], "adjoint_its": ast["fgmres_its_total"],
            "forward_advances": ast["forward_advances"]}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; --gpus must be 1 (multi-GPU sharding is a "
                                   "design note, not built)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2403_08084_amd as P
    import synth

    if args.calibrate_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    N = args.N
    n = (N - 1) ** 2
    tab = make_tableau(P, args.tableau)
    s = len(tab["b"])
    dt = args.dt
    kap = synth.grf_kappa(N, 1) if args.kappa == "grf" else np.ones(N * N)
    golden_ok = args.kappa == "grf" and dt == 1e-3  # the stored oracle result is for this workload
    u0, _ = synth.sine_modes_u0(N, 0)
    prob = P.Problem(N, torch.as_tensor(kap).cuda())
    u0d = torch.as_tensor(u0).cuda()
    prec = {"f32": P.F32, "bf16": P.BF16, "f64": P.F64}[args.precision]
    opts = solver_options(P, args)
    stp, u, ms, stats, setup_s = timed_run(P, torch, prob, tab, dt, u0d, args.steps, args.warmup, prec, opts)
    value = n * s * args.steps / (ms / 1e3)
    uh = u.cpu().numpy()
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
        "config": {"workload": f"diffusion Q1 {N}x{N}, "
                               + ("kappa=exp(GRF seed 1)" if args.kappa == "grf" else "kappa=1")
                               + f", {tab['name']}, dt={dt:g}, "
                               f"FGMRES({args.restart}) rtol 1e-10, " + (
                                   "1 monolithic GMG V-cycle Cheb(2)" if args.precond == "mmg" else
                                   f"P_{ {'gs': 'L', 'jacobi': 'D', 'rana': 'LD', 'gsu': 'U'}[args.precond]} + "
                                   "1 GMG V-cycle Cheb(2)") + f", MG {args.precision}"
                               + (", IA splitting" if args.splitting == "ia" else "")
                               + (", DIRK stage-by-stage solves" if args.stage_type == "dirk" else ""),
                   "N": N, "dofs": n, "stages": s},
        "fgmres_its_per_step": stats["fgmres_its_total"] / max(1, args.steps),
        "discarded_steps_per_step": stats["arnoldi_discarded"] / max(1, args.steps),
        "setup_s": setup_s,
        "solver": {"tableau": args.tableau, "stage_type": args.stage_type, "precond": args.precond,
                   "splitting": args.splitting, "orth": args.orth, "guess": args.guess,
                   "restart": args.restart,
                   "coarse_n": args.coarse_n},
        "error_vs_oracle": golden_error(uh, args.steps, args.tableau, golden_ok),
    }
    if not args.no_fp64 and prec != P.F64:
        _, u64, ms64, st64, _ = timed_run(P, torch, prob, tab, dt, u0d, args.steps, args.warmup, P.F64, opts)
        u64h = u64.cpu().numpy()
        out["fp64"] = {"value": n * s * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps,
                       "fgmres_its_per_step": st64["fgmres_its_total"] / max(1, args.steps),
                       "error_vs_oracle": golden_error(u64h, args.steps, args.tableau, golden_ok)}
        out["mixed_over_fp64"] = value / out["fp64"]["value"]
        out["rel_diff_mixed_vs_fp64"] = float(np.linalg.norm(uh - u64h) / np.linalg.norm(u64h))
    if not args.no_variants and args.tableau == "radau3" and args.stage_type == "coupled":
        # the same workload and accuracy target solved with the other stage preconditioners (mixed form)
        out["variants"] = {}
        for name, extra in (("P_LD, IA splitting", dict(precond=P.PC_RANA_LD, splitting=P.SPLIT_IA)),
                            ("monolithic MG", dict(precond=P.PC_MONOLITHIC, splitting=P.SPLIT_AI))):
            o2 = dict(opts)
            o2.update(extra)
            _, uv, msv, stv, _ = timed_run(P, torch, prob, tab, dt, u0d, args.steps, args.warmup, prec, o2)
            out["variants"][name] = {"value": n * s * args.steps / (msv / 1e3), "ms_per_step": msv / args.steps,
                                     "fgmres_its_per_step": stv["fgmres_its_total"] / max(1, args.steps),
                                     "error_vs_oracle": golden_error(uv.cpu().numpy(), args.steps, args.tableau, golden_ok)}
            del uv
    if not args.no_roofline:
        # same steps again with the measurement hook on the Gram-Schmidt pass (launched eagerly)
        stp.kernel_timer(0, True)
        u2 = u0d.clone()
        stp.advance(u2, args.steps)
        launches, kms, kbytes = stp.kernel_timer_read()
        stp.kernel_timer(0, False)
        achieved = kbytes / (kms / 1e3) / 1e9
        tb = traffic_bytes_per_launch() if args.orth == "dcgs2" else None
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                           "kernel": ("dots2_kernel + dcgs2_update_kernel (streaming Gram-Schmidt passes)"
                                      if args.orth == "dcgs2" else "ortho_kernel (streaming Gram-Schmidt pass)"),
                           "launches": launches,
                           "avg_us": 1e3 * kms / max(1, launches),
                           "algorithmic_bytes_per_launch": kbytes / max(1, launches),
                           "copy_ceiling": copy_ceiling(torch)}
    if not args.no_adjoint and not args.no_variants:
        out["adjoint"] = adjoint_timing(P, torch, synth)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
