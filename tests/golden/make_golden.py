#!/usr/bin/env python3
"""Write the full-size reference sketches used by the GPU parity tests and the benchmark.

Calls only the CPU oracle (oracle/) and the seeded input generators (synth/).
The full 1024^2 stage-coupled LU does not fit in memory, so the oracle's
eigen-decoupled direct tier (exact up to rounding, pinned against the coupled LU
at smaller sizes) produces the reference. Each stored vector u is summarised as
  * its 2-norm and max-norm,
  * the values at 1024 seeded indices,
  * 8 projections <g_k, u> onto seeded Gaussian vectors g_k (a sketch: for any
    error e, the projections are N(0, |e|^2) draws, so they bound |e|/|u|).
The sketch vectors are regenerated from their seed by the readers (sketch_vectors).

Usage: python tests/golden/make_golden.py [config4|config3|all]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SAMPLE_SEED = 12345
SKETCH_SEED = 54321
N_SAMPLES = 1024
N_SKETCH = 8


def sample_indices(n: int) -> np.ndarray:
    import synth

    return synth.sample_indices(n, N_SAMPLES, SAMPLE_SEED)


def sketch_vectors(n: int) -> np.ndarray:
    import synth

    return synth.sketch_vectors(n, N_SKETCH, SKETCH_SEED)


def summarise(u: np.ndarray, G: np.ndarray, idx: np.ndarray) -> dict:
    return {"norm2": float(np.linalg.norm(u)), "norminf": float(np.abs(u).max()),
            "samples": [float(v) for v in u[idx]], "sketch": [float(v) for v in G @ u]}


def run(name: str, tab_name: str, dt: float, nsteps: int, N: int = 1024, keep=(1, 20)):
    from oracle import step
    from oracle import tableaux as T
    import synth

    tab = {"radau3": T.radau_iia(3), "gl4": T.gauss_legendre(4)}[tab_name]
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    t0 = time.time()
    us = step.run(N, kap, tab, dt, nsteps, u0, tier="decoupled")
    elapsed = time.time() - t0
    n = (N - 1) ** 2
    idx = sample_indices(n)
    G = sketch_vectors(n)
    out = {
        "workload": f"{name}: Q1 {N}x{N}, kappa = exp(GRF seed 1, std 1, corr 0.1), u0 = 16 sine modes (seed 0), "
                    f"{tab['name']}, dt={dt}, {nsteps} steps",
        "oracle": "eigen-decoupled sparse direct (oracle.step.DecoupledLU), FP64",
        "N": N, "n": n, "dt": dt, "nsteps": nsteps, "tableau": tab_name,
        "sample_seed": SAMPLE_SEED, "sketch_seed": SKETCH_SEED, "n_samples": int(idx.size), "n_sketch": N_SKETCH,
        "indices": [int(i) for i in idx],
        "steps": {str(k): summarise(us[k], G, idx) for k in keep if k <= nsteps},
        "oracle_seconds": elapsed,
    }
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({elapsed:.1f} s)")


def run_adjoint(name: str = "config5_adjoint_512", N: int = 512, dt: float = 1e-3, nsteps: int = 40):
    """Oracle gradient of J = 1/2 |u_N - u_*|_M^2 with respect to log kappa (store-all reverse sweep)."""
    from oracle import adjoint, step
    from oracle import tableaux as T
    import synth

    tab = T.radau_iia(3)
    kap = synth.grf_kappa(N, 1)
    kref = synth.grf_kappa(N, 2)
    u0, _ = synth.sine_modes_u0(N, 0)
    t0 = time.time()
    ustar = step.run(N, kref, tab, dt, nsteps, u0)[-1]
    fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0)
    J, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    lam0, g = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, fwd=fwd)
    elapsed = time.time() - t0
    ne = N * N
    idx = synth.sample_indices(ne, N_SAMPLES, SAMPLE_SEED)
    G = synth.sketch_vectors(ne, N_SKETCH, SKETCH_SEED)
    n = (N - 1) ** 2
    idx_u = sample_indices(n)
    Gu = sketch_vectors(n)
    out = {
        "workload": f"{name}: Q1 {N}x{N}, kappa = exp(GRF seed 1), target from kappa_ref = exp(GRF seed 2), "
                    f"u0 = 16 sine modes (seed 0), RadauIIA(3), dt={dt}, {nsteps} steps, "
                    "J = 1/2 |u_N - u_*|_M^2, gradient w.r.t. per-element log kappa",
        "oracle": "coupled sparse LU forward and transposed solves (oracle.adjoint), FP64, all states stored",
        "N": N, "dt": dt, "nsteps": nsteps, "J": J,
        "sample_seed": SAMPLE_SEED, "sketch_seed": SKETCH_SEED, "n_samples": int(idx.size), "n_sketch": N_SKETCH,
        "grad_indices": [int(i) for i in idx], "grad": summarise(g, G, idx),
        "lam0_indices": [int(i) for i in idx_u], "lam0": summarise(lam0, Gu, idx_u),
        "uN": summarise(fwd[0][-1], Gu, idx_u), "ustar": summarise(ustar, Gu, idx_u),
        "oracle_seconds": elapsed,
    }
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({elapsed:.1f} s)")


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("config5", "all"):
        run_adjoint()
    if which in ("config4", "all"):
        run("config4_radau3_1024", "radau3", 1e-3, 20)
    if which in ("config3", "all"):
        run("config3_gl4_1024", "gl4", 5e-4, 20)


if __name__ == "__main__":
    main()
