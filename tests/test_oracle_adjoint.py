"""Pins for oracle.adjoint: dot-product test, finite differences, Taylor remainder."""
import numpy as np
import pytest

from oracle import adjoint, fem, step
from oracle import tableaux as T
import synth


@pytest.mark.parametrize("tab", [T.radau_iia(3), T.gauss_legendre(2), T.alexander()])
def test_step_map_dot_product(tab):
    N, dt = 12, 1e-2
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    sol = step.CoupledLU(M, K, tab["A"], dt)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, (N - 1) ** 2))
    lhs = adjoint.step_map(M, K, sol, tab, dt, x) @ y
    rhs = x @ adjoint.step_map_transpose(M, K, sol, tab, dt, y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def _J(N, logk, tab, dt, nsteps, u0, ustar):
    kap = np.exp(logk)
    us = step.run(N, kap, tab, dt, nsteps, u0)
    M, _ = fem.assemble(N, kap)
    return adjoint.objective(M, us[-1], ustar)[0]


def _setup(N=10, nsteps=4, dt=2e-3):
    tab = T.radau_iia(3)
    logk = synth.grf_log_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    ustar = step.run(N, np.exp(synth.grf_log_kappa(N, 2)), tab, dt, nsteps, u0)[-1]
    return tab, logk, u0, ustar


def test_gradient_central_differences():
    N, nsteps, dt = 10, 4, 2e-3
    tab, logk, u0, ustar = _setup(N, nsteps, dt)
    kap = np.exp(logk)
    fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0)
    _, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    lam0, g = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, fwd=fwd)
    dirs = synth.random_directions(4, N * N, seed=3)
    h = 1e-5
    for d in dirs:
        fd = (_J(N, logk + h * d, tab, dt, nsteps, u0, ustar) - _J(N, logk - h * d, tab, dt, nsteps, u0, ustar)) / (2 * h)
        assert abs(fd - g @ d) < 1e-7 * max(abs(fd), np.abs(g).sum() * 1e-3)
    # dJ/du0 as well
    du = synth.random_directions(1, (N - 1) ** 2, seed=5)[0]
    hu = 1e-4
    fdu = (_J(N, logk, tab, dt, nsteps, u0 + hu * du, ustar) - _J(N, logk, tab, dt, nsteps, u0 - hu * du, ustar)) / (2 * hu)
    assert abs(fdu - lam0 @ du) < 1e-8 * abs(fdu)


def test_gradient_taylor_remainder():
    # |J(theta + h d) - J(theta) - h g.d| = O(h^2): halving h quarters the remainder
    N, nsteps, dt = 8, 3, 5e-3
    tab, logk, u0, ustar = _setup(N, nsteps, dt)
    kap = np.exp(logk)
    fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0)
    _, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
    _, g = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, fwd=fwd)
    d = synth.random_directions(1, N * N, seed=7)[0]
    J0 = _J(N, logk, tab, dt, nsteps, u0, ustar)
    rem = []
    for h in (0.04, 0.02, 0.01):
        rem.append(abs(_J(N, logk + h * d, tab, dt, nsteps, u0, ustar) - J0 - h * (g @ d)))
    r1, r2 = rem[0] / rem[1], rem[1] / rem[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8


def test_decoupled_tier_gradient_equals_coupled():
    # the eigen-decoupled tier (used for the 512^2 gradient workload) gives the coupled LU's states, lam_0 and
    # gradient to rounding: its transposed solves are pinned here through the whole reverse sweep
    N, nsteps, dt = 10, 4, 2e-3
    tab, logk, u0, ustar = _setup(N, nsteps, dt)
    kap = np.exp(logk)
    res = {}
    for tier in ("coupled", "decoupled"):
        fwd = adjoint.forward(N, kap, tab, dt, nsteps, u0, tier=tier)
        J, lamN = adjoint.objective(fwd[2], fwd[0][-1], ustar)
        lam0, g = adjoint.gradient(N, kap, tab, dt, nsteps, u0, lamN, tier=tier, fwd=fwd)
        res[tier] = (fwd[0][-1], J, lam0, g)
    for a, b in zip(res["coupled"], res["decoupled"]):
        assert np.linalg.norm(np.atleast_1d(a) - np.atleast_1d(b)) < 1e-12 * np.linalg.norm(np.atleast_1d(a))
