"""GPU: a problem's kappa replaced in place and its stepper refreshed behaves exactly as a stepper built on the
new kappa (same estimates, same result bits); IrkSolve's cached solvers give the gradients of fresh ones, also
when two forward passes with different kappa come before their backward passes."""
import numpy as np
import pytest

import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make

pytestmark = pytest.mark.gpu


# 512^2 has five levels: the three-level DOWN/UP kernels, whose level diffusivities the refresh rebuilds, run too,
# and the monolithic cycle's finest level takes its large-tile kernels
@pytest.mark.parametrize("N,prec,pc,split", [(64, P.F32, P.PC_GS_LOWER, P.SPLIT_AI), (64, P.F64, P.PC_RANA_LD, P.SPLIT_AI),
                                             (64, P.BF16, P.PC_GS_LOWER, P.SPLIT_IA),
                                             (64, P.F32, P.PC_MONOLITHIC, P.SPLIT_AI),
                                             (512, P.F32, P.PC_GS_LOWER, P.SPLIT_AI),
                                             (512, P.F32, P.PC_MONOLITHIC, P.SPLIT_AI)])
def test_refresh_equals_a_new_stepper(N, prec, pc, split):
    dt, nsteps = 1e-3, 3
    k1, k2 = synth.grf_kappa(N, 1), synth.grf_kappa(N, 2)
    u0, _ = synth.sine_modes_u0(N, 0)
    opts = dict(mg_precision=prec, precond=pc, splitting=split, rtol=1e-10)
    prob, stp = make(N, k1, P.tableaux.radau_iia(3), dt, **opts)
    u = dev(u0)
    stp.advance(u, nsteps)  # graphs captured, previous-step state set, with kappa 1
    prob.set_kappa(dev(k2))
    stp.refresh()
    _, ref = make(N, k2, P.tableaux.radau_iia(3), dt, **opts)
    if pc == P.PC_MONOLITHIC:
        for tr in (False, True):
            for l in range(ref.mmg_levels - 1):
                assert stp.mmg_mu(l, tr) == ref.mmg_mu(l, tr)
    else:
        for i in range(3):
            for l in range(ref.levels - 1):
                assert stp.mu(i, l) == ref.mu(i, l)
    a, b = dev(u0), dev(u0)
    _, sa = stp.advance(a, nsteps)
    _, sb = ref.advance(b, nsteps)
    assert sa["fgmres_its_total"] == sb["fgmres_its_total"]
    assert np.array_equal(host(a), host(b))


def test_set_kappa_rejects_invalid_values_and_keeps_the_old():
    N = 32
    k1 = synth.grf_kappa(N, 1)
    prob, _ = make(N, k1, P.tableaux.radau_iia(2), 1e-3)
    x = dev(np.random.default_rng(3).standard_normal((N - 1) ** 2))
    y1 = host(prob.apply_stiffness(x))
    for bad in (0.0, -1.0, np.nan, np.inf):
        k = synth.grf_kappa(N, 2)
        k[5] = bad
        with pytest.raises(P.IrkError):
            prob.set_kappa(dev(k))
        assert np.array_equal(host(prob.apply_stiffness(x)), y1)


def _grads(cfg, u0, thetas, interleave):
    import torch

    out = []
    if interleave:
        ths = [dev(t).requires_grad_(True) for t in thetas]
        us = [P.IrkSolve.apply(dev(u0), th, cfg) for th in ths]
        sum((k + 1) * 0.5 * torch.dot(u, u) for k, u in enumerate(us)).backward()
        return [host(th.grad) for th in ths]
    for k, t in enumerate(thetas):
        th = dev(t).requires_grad_(True)
        u = P.IrkSolve.apply(dev(u0), th, cfg)
        ((k + 1) * 0.5 * torch.dot(u, u)).backward()
        out.append(host(th.grad))
    return out


def test_irk_solve_cache_matches_fresh_solvers():
    N, nsteps, dt = 32, 4, 1e-3
    u0, _ = synth.sine_modes_u0(N, 0)
    thetas = [np.log(synth.grf_kappa(N, s)) for s in (1, 2)]
    cfg = P.SolveConfig(N=N, tableau=P.tableaux.radau_iia(3), dt=dt, nsteps=nsteps, nsnap=2,
                        options={"rtol": 1e-13})
    fresh = []
    for k, t in enumerate(thetas):
        P._solver_cache.clear()
        fresh.append(_grads(cfg, u0, [t], False)[0] * (k + 1))
    P._solver_cache.clear()
    seq = _grads(cfg, u0, thetas, False)  # one cached solver, kappa reloaded for the second call
    assert len(P._solver_cache.entries) == 1
    solver = next(iter(P._solver_cache.entries.values()))
    assert solver.version == 1
    both = _grads(cfg, u0, thetas, True)  # two forward passes, then both backward passes
    assert next(iter(P._solver_cache.entries.values())) is solver
    for g, gs, gb in zip(fresh, seq, both):
        assert np.array_equal(gs, g)
        assert np.array_equal(gb, g)
