#!/usr/bin/env python3
"""Write the stored summary of the oracle's gradient for the 512^2 gradient workload (config 5), used by the GPU
parity test and the benchmark beside their whole-vector comparisons with the oracle computed in the run.

Calls only the CPU oracle (oracle/) and the seeded input generators (synth/). The gradient comes from the
oracle's coupled sparse LU (forward and transposed solves, all states stored), an independent tier from the
eigen-decoupled one the tests run live. Each stored vector u is summarised as
  * its 2-norm and max-norm,
  * the values at 1024 seeded indices,
  * 8 projections <g_k, u> onto seeded Gaussian vectors g_k (a sketch: for any
    error e, the projections are N(0, |e|^2) draws, so they bound |e|/|u|).
The sketch vectors are regenerated from their seed by the readers (sketch_vectors).

Usage: python tests/golden/make_golden.py
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
    run_adjoint()


if __name__ == "__main__":
    main()
