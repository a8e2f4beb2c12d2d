"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

Configs 3/4 (1024^2, variable kappa) are compared node by node with the oracle's eigen-decoupled direct solve
(oracle.step.DecoupledLU: the full coupled LU does not fit at 1024^2; the decoupled tier equals it to rounding,
pinned at smaller sizes), computed once per session: the relative L2 error of the whole interior vector at every
one of the 20 steps, maximised over the steps. Config 2 (512^2, kappa = 1) is compared with the closed form at
every step; config 5 (512^2 adjoint) with the oracle's whole gradient and lam_0 (decoupled direct tier, computed
once per session), with the summary of its coupled-LU gradient stored by tests/golden/make_golden.py and with
central finite differences."""
import json
import os
import time

import numpy as np
import pytest

from oracle import step
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_ORACLE = {}


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _compare(u, ref, idx, G):
    d = G @ u - np.asarray(ref["sketch"])
    sketch = float(np.sqrt(np.mean(d * d)) / ref["norm2"])
    samples = float(np.abs(u[idx] - np.asarray(ref["samples"])).max() / ref["norminf"])
    return max(sketch, samples, abs(np.linalg.norm(u) - ref["norm2"]) / ref["norm2"])


def _oracle_states(tname, dt, nsteps, N=1024):
    """[u^0 .. u^nsteps] of the workload (kappa = exp(GRF seed 1), 16 sine modes) from the decoupled direct tier."""
    key = (tname, dt, nsteps, N)
    if key not in _ORACLE:
        tab = {"radau3": OT.radau_iia(3), "gl4": OT.gauss_legendre(4)}[tname]
        t0 = time.time()
        _ORACLE[key] = step.run(N, synth.grf_kappa(N, 1), tab, dt, nsteps, synth.sine_modes_u0(N, 0)[0],
                                tier="decoupled")
        print(f"oracle {tname} {N}^2 {nsteps} steps: {time.time() - t0:.1f} s", flush=True)
    return _ORACLE[key]


def _run_fullsize(tname, tab, dt, nsteps, prec, pc, tol, N=1024, **opts):
    ref = _oracle_states(tname, dt, nsteps, N)
    kap = synth.grf_kappa(N, 1)
    _, stp = make(N, kap, tab, dt, mg_precision=prec, precond=pc, rtol=1e-10, **opts)
    u = dev(ref[0])
    errs = []
    for k in range(1, nsteps + 1):
        stp.advance(u, 1)
        errs.append(rel(host(u), ref[k]))
    print(f"{tname} prec {prec} pc {pc}: max over steps {max(errs):.2e}, final {errs[-1]:.2e}")
    assert max(errs) < tol, errs
    return errs


@pytest.mark.parametrize("prec,tol", [(P.F64, 1e-10), (P.F32, 1e-8), (P.BF16, 1e-8)])
def test_config4_fullsize(prec, tol):
    _run_fullsize("radau3", P.tableaux.radau_iia(3), 1e-3, 20, prec, P.PC_GS_LOWER, tol)


@pytest.mark.parametrize("pc,split", [(P.PC_RANA_LD, P.SPLIT_IA), (P.PC_MONOLITHIC, P.SPLIT_AI),
                                      (P.PC_MONOLITHIC, P.SPLIT_IA)])
def test_config4_fullsize_variants(pc, split):
    # the bench's variants of the mixed-precision workload: Rana-LD in the IA form and the monolithic cycle; the
    # IA form's unknowns are w = (A (x) I) k, but u^{n+1} is the same, so the same oracle states apply
    _run_fullsize("radau3", P.tableaux.radau_iia(3), 1e-3, 20, P.F32, pc, 1e-8, splitting=split)


@pytest.mark.parametrize("pc", [P.PC_JACOBI, P.PC_GS_LOWER])
def test_config3_fullsize_gl4(pc):
    _run_fullsize("gl4", P.tableaux.gauss_legendre(4), 5e-4, 20, P.F64, pc, 1e-10)


@pytest.mark.parametrize("prec,tol", [(P.F64, 1e-10), (P.F32, 1e-8)])
def test_dirk_fullsize(prec, tol):
    # the stage-by-stage path (one single-stage FGMRES per stage, known stages moved to the right) on the 1024^2
    # variable-kappa workload with the Alexander SDIRK(3), against the oracle's stage-by-stage direct tier
    N, dt, nsteps = 1024, 1e-3, 5
    key = ("dirk", N, dt, nsteps)
    if key not in _ORACLE:
        t0 = time.time()
        _ORACLE[key] = step.run(N, synth.grf_kappa(N, 1), OT.alexander(), dt, nsteps, synth.sine_modes_u0(N, 0)[0],
                                tier="dirk")
        print(f"oracle dirk {N}^2 {nsteps} steps: {time.time() - t0:.1f} s", flush=True)
    ref = _ORACLE[key]
    _, stp = make(N, synth.grf_kappa(N, 1), P.tableaux.alexander(), dt, mg_precision=prec, rtol=1e-11,
                  stage_type=P.STAGE_DIRK)
    u = dev(ref[0])
    errs = []
    for k in range(1, nsteps + 1):
        stp.advance(u, 1)
        errs.append(rel(host(u), ref[k]))
    print(f"dirk prec {prec}: max over steps {max(errs):.2e}")
    assert max(errs) < tol, errs


def test_config2_fullsize_closed_form():
    N, dt, nsteps = 512, 1e-3, 50
    u0, amps = synth.sine_modes_u0(N, 0)
    _, stp = make(N, np.ones(N * N), P.tableaux.radau_iia(3), dt, rtol=1e-10)
    cf = step.closed_form_modes(N, OT.radau_iia(3), dt, nsteps, amps)
    u = dev(u0)
    worst = 0.0
    for k in range(1, nsteps + 1):
        stp.advance(u, 1)
        worst = max(worst, rel(host(u), cf[k]))
    assert worst < 1e-10, worst


def _oracle_adjoint(N, dt, nsteps):
    """The oracle's gradient of config 5's objective from its eigen-decoupled direct tier (forward, target and
    transposed solves; about a minute on the host): (J, lam_0, grad)."""
    from oracle import adjoint

    key = ("adjoint", N, dt, nsteps)
    if key not in _ORACLE:
        tab = OT.radau_iia(3)
        kap = synth.grf_kappa(N, 1)
        u0, _ = synth.sine_modes_u0(N, 0)
        t0 = time.time()
        ustar = step.run(N, synth.grf_kappa(N, 2), tab, dt, nsteps, u0, tier="decoupled")[-1]
        fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0, tier="decoupled")
        J, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
        lam0, grad = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, tier="decoupled", fwd=fwd)
        print(f"oracle adjoint {N}^2 {nsteps} steps: {time.time() - t0:.1f} s", flush=True)
        _ORACLE[key] = (J, lam0, grad)
    return _ORACLE[key]


def test_config5_fullsize_adjoint():
    """Adjoint gradient at 512^2, 40 steps, 8 snapshots: the whole gradient and lam_0 against the oracle's
    (decoupled direct tier, 1e-8 relative L2), against the stored summary of the oracle's coupled-LU gradient
    written by tests/golden/make_golden.py, and against central finite differences.

    FD noise: J = 0.025 while |grad.d| ~ 6e-7 for a seeded unit direction d (the gradient is spread over 262,144
    elements), so J(theta +- h d) differ by ~1e-10 at h = 1e-4. Forward solves at rtol 2e-13 (the attainable
    FP64 residual of this operator is ~1.1e-13) perturb J by ~5e-14, i.e. ~3e-4 relative noise in the FD of a
    random direction; along the gradient direction (|grad.d| = |grad| ~ 3e-4) the noise is ~1e-6. Truncation
    error at h = 1e-4 is far below both."""
    import torch

    g = _load("config5_adjoint_512.json")
    N, dt, nsteps = g["N"], g["dt"], g["nsteps"]
    theta = synth.grf_log_kappa(N, 1)
    kref = synth.grf_kappa(N, 2)
    u0, _ = synth.sine_modes_u0(N, 0)
    tab = P.tableaux.radau_iia(3)
    opts = {"rtol": 2e-13}
    # target from the reference diffusivity
    _, sref = make(N, kref, tab, dt, **opts)
    ustar = dev(u0)
    sref.advance(ustar, nsteps)

    def J(th):
        prob, stp = make(N, np.exp(th), tab, dt, **opts)
        u = dev(u0)
        stp.advance(u, nsteps)
        d = u - ustar
        return 0.5 * float(torch.dot(d, prob.apply_mass(d))), (prob, stp, u)

    J0, (prob, stp, uN) = J(theta)
    assert abs(J0 - g["J"]) < 1e-9 * abs(g["J"])
    lamN = prob.apply_mass(uN - ustar)
    lam0, grad, st = stp.adjoint(dev(u0), nsteps, 8, lamN)
    assert st["forward_advances"] == 70  # optimal binomial schedule, 40 steps with 8 snapshots
    gh = host(grad)
    Jo, lam0o, grado = _oracle_adjoint(N, dt, nsteps)
    eg, el = rel(gh, grado), rel(host(lam0), lam0o)
    print(f"config 5: J {J0:.15e} (oracle {Jo:.15e}), gradient rel L2 {eg:.2e}, lam_0 rel L2 {el:.2e}")
    assert abs(J0 - Jo) < 1e-9 * abs(Jo) and eg < 1e-8 and el < 1e-8
    idx = np.asarray(g["grad_indices"])
    G = synth.sketch_vectors(N * N, g["n_sketch"], g["sketch_seed"])
    assert _compare(gh, g["grad"], idx, G) < 1e-8
    Gu = synth.sketch_vectors((N - 1) ** 2, g["n_sketch"], g["sketch_seed"])
    assert _compare(host(lam0), g["lam0"], np.asarray(g["lam0_indices"]), Gu) < 1e-8
    h = 1e-4

    def fd(d):
        return (J(theta + h * d)[0] - J(theta - h * d)[0]) / (2 * h)

    dg = gh / np.linalg.norm(gh)
    assert abs(fd(dg) - gh @ dg) < 1e-5 * abs(gh @ dg)
    worst = 0.0
    for d in synth.random_directions(32, N * N, seed=3):
        worst = max(worst, abs(fd(d) - gh @ d) / abs(gh @ d))
    assert worst < 5e-3, worst
