"""Discrete adjoint of the Runge-Kutta time-step map and the log-diffusivity gradient (FP64, CPU).

Test infrastructure only (see the package docstring).

The paper does not treat adjoints; this is the standard discrete adjoint of the
linear step map of Section 2 / eq:block_struct_AI, derived here. With F = 0 and
theta_e = log kappa_e, one step is

    Acal k_n = -(1 (x) K) u_n,     u_{n+1} = u_n + dt (b^T (x) I) k_n,
    Acal = I (x) M + dt A (x) K.

For J(u_N) with lambda_N = dJ/du_N the reverse sweep n = N-1 .. 0 is

    Acal^T nu_n = dt (b (x) lambda_{n+1}),            (Acal^T = I (x) M + dt A^T (x) K)
    lambda_n   = lambda_{n+1} - K sum_i nu_{n,i},
    dJ/dtheta_e -= kappa_e sum_i (nu_{n,i}|_e)^T Ke_ref (U_{n,i}|_e),
                   U_{n,i} = u_n + dt sum_j a_ij k_{n,j},

where Ke_ref is the kappa = 1 element stiffness matrix and |_e gathers the four
nodal values of element e (boundary values are zero). The gradient term follows
from differentiating both K occurrences of the step (dK/dtheta_e = kappa_e Ke_ref
scattered to the element's nodes).
"""
from __future__ import annotations

import numpy as np

from . import fem
from .step import CoupledLU, DecoupledLU, stage_rhs, update


def _solver(M, K, A, dt, tier):
    if tier == "coupled":
        return CoupledLU(M, K, A, dt)
    if tier == "decoupled":
        return DecoupledLU(M, K, A, dt)
    raise ValueError(tier)


def objective(M, uN, ustar):
    """J = 1/2 (u_N - u_*)^T M (u_N - u_*) and its gradient M (u_N - u_*)."""
    d = uN - ustar
    Md = M @ d
    return 0.5 * float(d @ Md), Md


def forward(N, kappa, tab, dt, nsteps, u0, tier="coupled"):
    """Forward sweep storing every state and stage block: (us, ks, M, K, solver)."""
    M, K = fem.assemble(N, kappa)
    A = np.asarray(tab["A"])
    b = np.asarray(tab["b"])
    s = b.size
    sol = _solver(M, K, A, dt, tier)
    us = [np.asarray(u0, dtype=np.float64).copy()]
    ks = []
    for _ in range(nsteps):
        k = sol.solve(stage_rhs(K, us[-1], s))
        ks.append(k)
        us.append(update(us[-1], k, b, dt))
    return us, ks, M, K, sol


def gradient(N, kappa, tab, dt, nsteps, u0, lam_N, tier="coupled", fwd=None):
    """Reverse sweep with every forward state stored.

    Returns (lambda_0, g) with lambda_0 = dJ/du_0 and g = dJ/dlog(kappa) (element layout).
    """
    A = np.asarray(tab["A"])
    b = np.asarray(tab["b"])
    s = b.size
    if fwd is None:
        fwd = forward(N, kappa, tab, dt, nsteps, u0, tier)
    us, ks, M, K, sol = fwd
    kap = np.asarray(kappa, dtype=np.float64) if kappa is not None else np.ones(N * N)
    Ke_ref, _ = fem.element_matrices(1.0 / N)
    lam = np.asarray(lam_N, dtype=np.float64).copy()
    g = np.zeros(N * N)
    n = lam.size
    for step in range(nsteps - 1, -1, -1):
        nu = sol.solve(dt * np.kron(b, lam), trans=True).reshape(s, n)
        kk = ks[step].reshape(s, n)
        for i in range(s):
            Ui = us[step] + dt * (A[i] @ kk)
            nu_e = fem.element_gather(N, nu[i])
            U_e = fem.element_gather(N, Ui)
            g -= kap * np.einsum("ea,ab,eb->e", nu_e, Ke_ref, U_e)
        lam = lam - K @ nu.sum(axis=0)
    return lam, g


def step_map(M, K, sol, tab, dt, x):
    """One forward step S x (F = 0)."""
    b = np.asarray(tab["b"])
    k = sol.solve(stage_rhs(K, x, b.size))
    return update(x, k, b, dt)


def step_map_transpose(M, K, sol, tab, dt, y):
    """S^T y = y - K sum_i nu_i with Acal^T nu = dt (b (x) y)."""
    b = np.asarray(tab["b"])
    s = b.size
    nu = sol.solve(dt * np.kron(b, y), trans=True).reshape(s, -1)
    return y - K @ nu.sum(axis=0)
