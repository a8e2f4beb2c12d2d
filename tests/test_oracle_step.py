"""Pins for oracle.step: closed forms, brute force, tier agreement, invariants."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, step
from oracle import tableaux as T
import synth


def _pade_radau2(z):
    return (1 + z / 3) / (1 - 2 * z / 3 + z * z / 6)


def _lam(N, j, k):
    h = 1.0 / N
    one = lambda m: 6 / h**2 * (1 - np.cos(m * np.pi * h)) / (2 + np.cos(m * np.pi * h))  # noqa: E731
    return one(j) + one(k)


def test_config1_decay_closed_form():
    # 32x32, Radau IIA(2), dt = 1/32, 10 steps, u0 = sin(pi x) sin(pi y): u10 = R(-dt lam11)^10 u0
    N, dt = 32, 1.0 / 32
    u0 = synth.sine_mode_vector(N, 1, 1)
    us = step.run(N, None, T.radau_iia_printed(2), dt, 10, u0)
    R = _pade_radau2(-dt * _lam(N, 1, 1))
    assert abs(R**10 - 0.0020475389) < 1e-10
    for n in range(11):
        assert np.linalg.norm(us[n] - R**n * u0) <= 1e-12 * np.linalg.norm(R**n * u0)


def _stage_residual(M, K, A, dt, u, k):
    """Residual of the stage equations written stage by stage (eq:rkheat form)."""
    s = A.shape[0]
    kk = k.reshape(s, -1)
    res = []
    for i in range(s):
        Ui = u + dt * sum(A[i, j] * kk[j] for j in range(s))
        res.append(M @ kk[i] + K @ Ui)
    return np.concatenate(res)


@pytest.mark.parametrize("tabname", ["radau2", "radau3", "gl4", "lobatto", "alexander", "wso433"])
def test_dense_and_coupled_lu_solve_stage_equations(tabname):
    tab = {"radau2": T.radau_iia(2), "radau3": T.radau_iia(3), "gl4": T.gauss_legendre(4),
           "lobatto": T.lobatto_iiic2(), "alexander": T.alexander(), "wso433": T.wsodirk433()}[tabname]
    N, dt = 6, 0.01
    kap = synth.grf_kappa(N, 11)
    M, K = fem.assemble(N, kap)
    A = tab["A"]
    rng = np.random.default_rng(1)
    u = rng.standard_normal((N - 1) ** 2)
    rhs = step.stage_rhs(K, u, A.shape[0])
    kd = step.dense_solve(M, K, A, dt, rhs)
    kc = step.CoupledLU(M, K, A, dt).solve(rhs)
    assert np.abs(_stage_residual(M, K, A, dt, u, kd)).max() < 1e-12
    assert np.linalg.norm(kc - kd) < 1e-12 * np.linalg.norm(kd)


@pytest.mark.parametrize("tab", [T.radau_iia(3), T.gauss_legendre(4)])
def test_decoupled_matches_coupled(tab):
    N, dt = 32, 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal(tab["b"].size * (N - 1) ** 2)
    c = step.CoupledLU(M, K, tab["A"], dt)
    d = step.DecoupledLU(M, K, tab["A"], dt)
    for trans in (False, True):
        x1, x2 = c.solve(rhs, trans), d.solve(rhs, trans)
        assert np.linalg.norm(x1 - x2) < 1e-12 * np.linalg.norm(x1)
    # the transpose solve really solves with I (x) M + dt A^T (x) K
    At = step.coupled_matrix(M, K, tab["A"].T, dt)
    x = c.solve(rhs, True)
    assert np.linalg.norm(At @ x - rhs) < 1e-12 * np.linalg.norm(rhs)


def test_closed_form_any_matches_coupled():
    N, dt, n = 24, 2e-3, 5
    u0 = synth.white_noise_u0(N, 4)
    tab = T.radau_iia(3)
    us = step.run(N, None, tab, dt, n, u0)
    cf = step.closed_form_any(N, tab, dt, n, u0)
    assert np.linalg.norm(us[-1] - cf) < 1e-12 * np.linalg.norm(cf)


def test_closed_form_modes_matches_coupled():
    N, dt, n = 32, 1e-3, 4
    u0, amps = synth.sine_modes_u0(N, 0)
    tab = T.radau_iia(3)
    us = step.run(N, None, tab, dt, n, u0)
    cf = step.closed_form_modes(N, tab, dt, n, amps)
    for a, b in zip(us, cf):
        assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(b)


def test_stiffly_accurate_last_stage_value():
    # Radau IIA is stiffly accurate (b = last row of A), so u^{n+1} equals the last stage value
    N, dt = 16, 5e-3
    kap = synth.grf_kappa(N, 3)
    tab = T.radau_iia(3)
    us, ks = step.run(N, kap, tab, dt, 1, synth.white_noise_u0(N, 4), return_stages=True)
    kk = ks[0].reshape(3, -1)
    Us = us[0] + dt * (tab["A"][2] @ kk)
    assert np.linalg.norm(Us - us[1]) < 1e-14 * np.linalg.norm(us[1])


def test_backward_euler_textbook():
    # s = 1, A = [[1]]: (M + dt K) u^{n+1} = M u^n
    N, dt = 16, 1e-2
    kap = synth.grf_kappa(N, 3)
    M, K = fem.assemble(N, kap)
    u0 = synth.white_noise_u0(N, 4)
    us = step.run(N, kap, T.backward_euler(), dt, 1, u0)
    ref = spla.spsolve((M + dt * K).tocsc(), M @ u0)
    assert np.linalg.norm(us[1] - ref) < 1e-13 * np.linalg.norm(ref)


def test_dirk_sequential_solve():
    # a lower-triangular A decouples the stages: s consecutive single-stage solves (Section 2.3)
    N, dt = 12, 1e-2
    kap = synth.grf_kappa(N, 3)
    M, K = fem.assemble(N, kap)
    tab = T.alexander()
    A = tab["A"]
    u = synth.white_noise_u0(N, 4)
    k = step.CoupledLU(M, K, A, dt).solve(step.stage_rhs(K, u, 3))
    kk = []
    for i in range(3):
        r = -(K @ (u + dt * sum(A[i, j] * kk[j] for j in range(i))))
        kk.append(spla.spsolve((M + dt * A[i, i] * K).tocsc(), r))
    assert np.linalg.norm(k - np.concatenate(kk)) < 1e-12 * np.linalg.norm(k)
    # the oracle's stage-by-stage tier, forward and transposed, against the coupled LU
    assert np.linalg.norm(step.dirk_solve(M, K, A, dt, step.stage_rhs(K, u, 3)) - k) < 1e-12 * np.linalg.norm(k)
    f = np.random.default_rng(8).standard_normal(3 * (N - 1) ** 2)
    kt = step.CoupledLU(M, K, A, dt).solve(f, trans=True)
    assert np.linalg.norm(step.dirk_solve(M, K, A, dt, f, trans=True) - kt) < 1e-12 * np.linalg.norm(kt)
    # with one factorisation kept per diagonal entry (the form the run tier uses), forward and transposed, on a
    # tableau whose diagonal entries differ too; the second round reuses the kept factors
    for tab2 in (tab, T.wsodirk433()):
        A2 = tab2["A"]
        s2 = A2.shape[0]
        f2 = np.random.default_rng(9).standard_normal(s2 * (N - 1) ** 2)
        k2 = step.CoupledLU(M, K, A2, dt).solve(step.stage_rhs(K, u, s2))
        kt2 = step.CoupledLU(M, K, A2, dt).solve(f2, trans=True)
        lu = {}
        for _ in range(2):
            r = step.dirk_solve(M, K, A2, dt, step.stage_rhs(K, u, s2), lu=lu)
            assert np.linalg.norm(r - k2) < 1e-12 * np.linalg.norm(k2)
            rt = step.dirk_solve(M, K, A2, dt, f2, trans=True, lu=lu)
            assert np.linalg.norm(rt - kt2) < 1e-12 * np.linalg.norm(kt2)
        assert len(lu) == len(set(np.diag(A2)))
    with pytest.raises(ValueError):
        step.dirk_solve(M, K, T.radau_iia(2)["A"], dt, f[: 2 * (N - 1) ** 2])


@pytest.mark.parametrize("tabname", ["alexander", "wso433"])
def test_dirk_tier_matches_closed_form(tabname):
    # kappa = 1, sine modes: u_n = sum alpha_jk R(-dt lam_jk)^n phi_jk with R of the DIRK tableau
    tab = {"alexander": T.alexander(), "wso433": T.wsodirk433()}[tabname]
    N, dt, nsteps = 16, 1e-2, 5
    u0, amps = synth.sine_modes_u0(N, 0)
    us = step.run(N, None, tab, dt, nsteps, u0, tier="dirk")
    cf = step.closed_form_modes(N, tab, dt, nsteps, amps)
    for n in range(nsteps + 1):
        assert np.linalg.norm(us[n] - cf[n]) <= 1e-12 * np.linalg.norm(cf[n])


# ---------------------------------------------------------------- IA splitting (eq:butcherw, eq:block_struct_IA)


def test_ia_config1_decay_closed_form():
    # the IA form is a change of unknowns only: config 1 still decays as R(-dt lam11)^n
    N, dt = 32, 1.0 / 32
    u0 = synth.sine_mode_vector(N, 1, 1)
    us = step.run(N, None, T.radau_iia_printed(2), dt, 10, u0, splitting="IA")
    R = _pade_radau2(-dt * _lam(N, 1, 1))
    for n in range(11):
        assert np.linalg.norm(us[n] - R**n * u0) <= 1e-12 * np.linalg.norm(R**n * u0)


@pytest.mark.parametrize("tabname", ["radau3", "gl4", "lobatto", "alexander"])
def test_ia_unknowns_are_stage_combinations(tabname):
    # w_i = sum_j a_ij k_j (eq:butcherw) and both forms give the same step, for any invertible A
    tab = {"radau3": T.radau_iia(3), "gl4": T.gauss_legendre(4), "lobatto": T.lobatto_iiic2(),
           "alexander": T.alexander()}[tabname]
    N, dt = 12, 2e-2
    kap = synth.grf_kappa(N, 3)
    u0 = synth.white_noise_u0(N, 4)
    A = tab["A"]
    s = A.shape[0]
    ua, ka = step.run(N, kap, tab, dt, 3, u0, return_stages=True)
    ui, wi = step.run(N, kap, tab, dt, 3, u0, return_stages=True, splitting="IA")
    ud = step.run(N, kap, tab, dt, 3, u0, tier="dense", splitting="IA")
    for n in range(1, 4):
        assert np.linalg.norm(ui[n] - ua[n]) < 1e-13 * np.linalg.norm(ua[n])
        assert np.linalg.norm(ud[n] - ua[n]) < 1e-13 * np.linalg.norm(ua[n])
        k = ka[n - 1].reshape(s, -1)
        w = np.stack([sum(A[i, j] * k[j] for j in range(s)) for i in range(s)])
        assert np.linalg.norm(wi[n - 1] - w.ravel()) < 1e-12 * np.linalg.norm(w)


def test_ia_stage_equations_written_out():
    # eq:stageeqw for the heat equation: sum_j (A^{-1})_ij M w_j + K (u + dt w_i) = 0 stage by stage
    N, dt = 10, 1e-2
    kap = synth.grf_kappa(N, 5)
    M, K = fem.assemble(N, kap)
    tab = T.radau_iia(3)
    u0 = synth.white_noise_u0(N, 6)
    _, ws = step.run(N, kap, tab, dt, 1, u0, return_stages=True, splitting="IA")
    W = ws[0].reshape(3, -1)
    Ainv = np.linalg.inv(tab["A"])
    for i in range(3):
        r = sum(Ainv[i, j] * (M @ W[j]) for j in range(3)) + K @ (u0 + dt * W[i])
        assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(K @ u0)


def test_ia_stiffly_accurate_update_is_last_w():
    # Radau IIA: b^T A^{-1} = e_s^T, so u^{n+1} = u^n + dt w_s
    N, dt = 16, 5e-3
    kap = synth.grf_kappa(N, 3)
    u0 = synth.white_noise_u0(N, 4)
    us, ws = step.run(N, kap, T.radau_iia(3), dt, 1, u0, return_stages=True, splitting="IA")
    assert np.linalg.norm(us[0] + dt * ws[0].reshape(3, -1)[2] - us[1]) < 1e-14 * np.linalg.norm(us[1])
