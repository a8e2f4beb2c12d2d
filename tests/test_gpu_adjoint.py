"""GPU parity: discrete adjoint (a8) with binomial checkpointing (a9) vs the oracle's store-all gradient."""
import numpy as np
import pytest

from oracle import adjoint, fem, step
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu


def _setup(N, nsteps, dt):
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    ustar = step.run(N, synth.grf_kappa(N, 2), OT.radau_iia(3), dt, nsteps, u0)[-1]
    return kap, u0, ustar


@pytest.mark.parametrize("nsnap,split,pc", [(2, P.SPLIT_AI, P.PC_GS_LOWER), (3, P.SPLIT_AI, P.PC_GS_LOWER),
                                            (100, P.SPLIT_AI, P.PC_GS_LOWER), (3, P.SPLIT_AI, P.PC_RANA_LD),
                                            (3, P.SPLIT_IA, P.PC_GS_LOWER), (3, P.SPLIT_IA, P.PC_RANA_LD),
                                            (3, P.SPLIT_AI, P.PC_MONOLITHIC)])
def test_adjoint_matches_oracle(nsnap, split, pc):
    # the gradient of the discrete step map does not depend on the stage formulation or the preconditioner
    N, nsteps, dt = 32, 6, 1e-3
    kap, u0, ustar = _setup(N, nsteps, dt)
    fwd = adjoint.forward(N, kap, OT.radau_iia(3), dt, nsteps, u0)
    _, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    lam0_o, g_o = adjoint.gradient(N, kap, OT.radau_iia(3), dt, nsteps, u0, lamN, fwd=fwd)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-13, splitting=split, precond=pc)
    lam0, g, st = stp.adjoint(dev(u0), nsteps, nsnap, dev(lamN))
    assert rel(host(lam0), lam0_o) < 1e-9
    assert rel(host(g), g_o) < 1e-9
    from oracle import revolve
    assert st["forward_advances"] == revolve.min_advances_dp(nsteps, min(nsnap, nsteps))


def test_dirk_adjoint_matches_oracle():
    # stage-by-stage forward solves and backward (transposed) stage solves for WSODIRK433
    N, nsteps, dt = 32, 5, 1e-3
    kap, u0, ustar = _setup(N, nsteps, dt)
    tab = OT.wsodirk433()
    fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0)
    _, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    lam0_o, g_o = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, fwd=fwd)
    _, stp = make(N, kap, P.tableaux.wsodirk433(), dt, rtol=1e-13, stage_type=P.STAGE_DIRK)
    lam0, g, st = stp.adjoint(dev(u0), nsteps, 2, dev(lamN))
    assert rel(host(lam0), lam0_o) < 1e-9
    assert rel(host(g), g_o) < 1e-9


def test_revolve_equals_store_all_bitwise():
    N, nsteps, dt = 32, 7, 1e-3
    kap, u0, ustar = _setup(N, nsteps, dt)
    lamN = np.random.default_rng(1).standard_normal((N - 1) ** 2)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-12)
    a = stp.adjoint(dev(u0), nsteps, 3, dev(lamN))
    b = stp.adjoint(dev(u0), nsteps, nsteps, dev(lamN))
    assert np.array_equal(host(a[0]), host(b[0]))
    assert np.array_equal(host(a[1]), host(b[1]))


def test_revolve_schedule_is_optimal_and_consistent():
    from oracle import revolve

    for l in (1, 2, 5, 13, 40):
        for c in (1, 2, 3, 8):
            acts, adv = P.revolve_schedule(l, c)
            assert adv == revolve.min_advances_dp(l, min(c, l))
            # replay: every step reversed once, in decreasing order, from the right state
            cur, slots, rev = 0, {}, []
            for kind, arg in acts:
                if kind == 0:
                    cur += arg
                elif kind == 1:
                    slots[arg] = cur
                elif kind == 2:
                    cur = slots[arg]
                else:
                    assert arg == cur
                    rev.append(arg)
            assert rev == list(range(l - 1, -1, -1))
            assert max(slots) < max(1, min(c, l))


def test_autograd_function_fd():
    import torch

    N, nsteps, dt = 16, 4, 2e-3
    kap, u0, ustar = _setup(N, nsteps, dt)
    cfg = P.SolveConfig(N=N, tableau=P.tableaux.radau_iia(3), dt=dt, nsteps=nsteps, nsnap=2, options={"rtol": 1e-14})
    theta = dev(np.log(kap)).requires_grad_(True)
    u0t = dev(u0).requires_grad_(True)
    M, _ = fem.assemble(N, kap)
    Md = dev(M.toarray())
    us = dev(ustar)

    def J(th, uu):
        uN = P.IrkSolve.apply(uu, th, cfg)
        d = uN - us
        return 0.5 * torch.dot(d, Md @ d)

    j = J(theta, u0t)
    j.backward()
    d = dev(synth.random_directions(1, N * N, seed=3)[0])
    h = 1e-5
    with torch.no_grad():
        fd = (J(theta + h * d, u0t) - J(theta - h * d, u0t)) / (2 * h)
    assert abs(float(fd) - float(torch.dot(theta.grad, d))) < 1e-6 * abs(float(fd)) + 1e-14
