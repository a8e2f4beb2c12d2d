"""Pins for oracle.mg: transfers, Galerkin identity, Chebyshev polynomial, V-cycle, preconditioners."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, mg, step
from oracle import tableaux as T
import synth


def test_splitmix64_reference_value():
    # first outputs of SplitMix64 seeded with 0 (state advanced before mixing)
    assert mg.splitmix64(0) == 0xE220A8397B1DCDAF
    assert mg.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    v = mg.start_vector(4, 2)
    ref = [2 * ((mg.splitmix64((2 << 32) + p) >> 11) / 2.0**53) - 1 for p in range(4)]
    assert np.array_equal(v, np.array(ref))


def test_level_sizes():
    assert mg.level_sizes(1024, 8) == [1024, 512, 256, 128, 64, 32, 16, 8]
    assert mg.level_sizes(1024) == [1024, 512, 256, 128, 64, 32]
    assert mg.level_sizes(96, 8) == [96, 48, 24, 12, 6]
    assert mg.level_sizes(96) == [96, 48, 24]
    assert mg.level_sizes(8) == [8]
    assert mg.level_sizes(33) == [33]


def test_prolongation_is_bilinear_interpolation():
    Nc = 6
    rng = np.random.default_rng(0)
    ec = rng.standard_normal((Nc - 1) ** 2)
    E = np.zeros((Nc + 1, Nc + 1))
    E[1:Nc, 1:Nc] = ec.reshape(Nc - 1, Nc - 1)
    Nf = 2 * Nc
    ref = np.zeros((Nf - 1, Nf - 1))
    for j in range(1, Nf):
        for i in range(1, Nf):
            X, Y = i / 2.0, j / 2.0  # coarse coordinates
            I0, J0 = min(int(X), Nc - 1), min(int(Y), Nc - 1)
            fx, fy = X - I0, Y - J0
            ref[j - 1, i - 1] = ((1 - fx) * (1 - fy) * E[J0, I0] + fx * (1 - fy) * E[J0, I0 + 1]
                                 + fx * fy * E[J0 + 1, I0 + 1] + (1 - fx) * fy * E[J0 + 1, I0])
    assert np.abs(mg.prolongation(Nc) @ ec - ref.ravel()).max() < 1e-15


def test_galerkin_identity_nested_spaces():
    # With kappa constant on each coarse element, P^T K_h P = K_H and P^T M_h P = M_H exactly
    Nc = 8
    kc = synth.grf_kappa(Nc, 9)
    kf = np.repeat(np.repeat(kc.reshape(Nc, Nc), 2, axis=0), 2, axis=1).ravel()
    assert np.abs(mg.coarsen_kappa(2 * Nc, kf) - kc).max() < 1e-15
    Mf, Kf = fem.assemble(2 * Nc, kf)
    Mc, Kc = fem.assemble(Nc, kc)
    P = mg.prolongation(Nc)
    assert abs(P.T @ Kf @ P - Kc).max() < 1e-13
    assert abs(P.T @ Mf @ P - Mc).max() < 1e-16


def test_chebyshev_error_polynomial():
    # error propagation of the Jacobi-Chebyshev smoother on a generalized eigenvector
    # (B v = lam D v) is T_d((theta - lam)/delta) / T_d(theta/delta)
    N = 8
    kap = synth.grf_kappa(N, 2)
    M, K = fem.assemble(N, kap)
    B = (M + 0.01 * K).tocsr()
    D = B.diagonal()
    lam, V = sla.eigh(B.toarray(), np.diag(D))
    lo, hi = 0.25 * lam.max(), 1.1 * lam.max()
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    for deg in (1, 2, 3):
        Td = np.polynomial.chebyshev.Chebyshev.basis(deg)
        for idx in (0, 7, 20, len(lam) - 1):
            v = V[:, idx]
            # smoothing B x = 0 from x0 = v: the iterate is the propagated error
            e = mg.chebyshev_smooth(B, 1.0 / D, np.zeros_like(v), v, lo, hi, deg)
            fac = Td((theta - lam[idx]) / delta) / Td(theta / delta)
            assert np.linalg.norm(e - fac * v) < 1e-12 * np.linalg.norm(v)


def test_power_mu_estimate():
    N = 16
    kap = synth.grf_kappa(N, 2)
    M, K = fem.assemble(N, kap)
    B = (M + 1e-3 * K).tocsr()
    Dinv = 1.0 / B.diagonal()
    lmax = sla.eigh(B.toarray(), np.diag(1.0 / Dinv), eigvals_only=True).max()
    mu = mg.power_mu(B, Dinv, 0, 15)
    assert mu <= lmax * (1 + 1e-12)
    assert mu >= 0.8 * lmax


def test_single_level_vcycle_is_exact():
    N = 8
    kap = synth.grf_kappa(N, 2)
    h = mg.Hierarchy(N, kap, 1e-3, coarse_n=8)
    assert h.sizes == [8]
    M, K = fem.assemble(N, kap)
    t = np.random.default_rng(0).standard_normal((N - 1) ** 2)
    x = h.vcycle(0.3, t)
    assert np.linalg.norm((M + 1e-3 * 0.3 * K) @ x - t) < 1e-14 * np.linalg.norm(t)


def test_vcycle_symmetric_and_contracting():
    N = 64
    kap = synth.grf_kappa(N, 1)
    dt, a = 1e-3, 0.2
    hier = mg.Hierarchy(N, kap, dt, coarse_n=8)
    M, K = fem.assemble(N, kap)
    B = (M + dt * a * K).tocsr()
    rng = np.random.default_rng(3)
    u, w = rng.standard_normal((2, (N - 1) ** 2))
    assert abs(u @ hier.vcycle(a, w) - w @ hier.vcycle(a, u)) < 1e-10 * abs(u @ hier.vcycle(a, w))
    e = rng.standard_normal((N - 1) ** 2)
    for _ in range(3):
        e2 = e - hier.vcycle(a, B @ e)
        assert np.linalg.norm(e2) < 0.2 * np.linalg.norm(e)
        e = e2


def _block_prec_matrix(M, K, Atil, dt):
    return step.coupled_matrix(M, K, Atil, dt)


def test_ldu_factorisation():
    for A in (T.radau_iia(3)["A"], T.gauss_legendre(4)["A"], T.lobatto_iiic2()["A"]):
        L1, D, U1 = mg.ldu(A)
        assert np.abs(L1 @ np.diag(D) @ U1 - A).max() < 1e-15
        assert np.array_equal(np.diag(L1), np.ones(len(D))) and np.array_equal(np.diag(U1), np.ones(len(D)))
        assert np.abs(np.triu(L1, 1)).max() == 0 and np.abs(np.tril(U1, -1)).max() == 0
        assert np.all(D > 0)
    # a lower-triangular A (a DIRK) is its own L1 D, so Rana-LD reproduces the stage operator
    A = T.alexander()["A"]
    assert np.abs(mg.preconditioner_matrix("rana_ld", A) - A).max() < 1e-15
    # first pivot and the 2x2 Schur complement by hand
    A2 = np.array([[2.0, 1.0], [4.0, 5.0]])
    L1, D, U1 = mg.ldu(A2)
    assert D[0] == 2.0 and D[1] == 5.0 - 4.0 * 1.0 / 2.0 and L1[1, 0] == 2.0 and U1[0, 1] == 0.5


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("kind", ["jacobi", "gs_lower", "gs_upper", "rana_ld"])
def test_exact_block_preconditioner_definition(kind, trans):
    # with exact blocks, P^{-1} v solves I (x) M + dt Atil (x) K with Atil = D, L + D or L1 D; the transposed
    # system's preconditioner is the transpose of that matrix
    N, dt = 10, 1e-2
    kap = synth.grf_kappa(N, 4)
    M, K = fem.assemble(N, kap)
    A = T.radau_iia(3)["A"]
    L1, D, U1 = mg.ldu(A)
    Atil = {"jacobi": np.diag(np.diag(A)), "gs_lower": np.tril(A), "gs_upper": np.triu(A),
            "rana_ld": L1 @ np.diag(D)}[kind]
    v = np.random.default_rng(5).standard_normal(3 * (N - 1) ** 2)
    z = mg.apply_block_preconditioner(kind, A, dt, K, v, mg.exact_block_solver(M, K, Atil, dt), trans=trans)
    P = _block_prec_matrix(M, K, Atil, dt)
    if trans:
        P = P.T
    assert np.linalg.norm(P @ z - v) < 1e-12 * np.linalg.norm(v)


def test_gs_lower_is_exact_for_dirk():
    # lower-triangular A: P_L equals the stage-coupled operator itself (Section 2.3)
    N, dt = 10, 1e-2
    kap = synth.grf_kappa(N, 4)
    M, K = fem.assemble(N, kap)
    A = T.alexander()["A"]
    Acal = step.coupled_matrix(M, K, A, dt)
    x = np.random.default_rng(6).standard_normal(3 * (N - 1) ** 2)
    z = mg.apply_block_preconditioner("gs_lower", A, dt, K, Acal @ x, mg.exact_block_solver(M, K, A, dt))
    assert np.linalg.norm(z - x) < 1e-12 * np.linalg.norm(x)
    # and the block upper variant is exact for the transposed system (A^T upper triangular): backward substitution
    AcalT = step.coupled_matrix(M, K, A.T, dt)
    zt = mg.apply_block_preconditioner("gs_upper", A.T, dt, K, AcalT @ x, mg.exact_block_solver(M, K, A, dt))
    assert np.linalg.norm(zt - x) < 1e-12 * np.linalg.norm(x)
    # P_LD is exact for a DIRK too: A = L1 D with U1 = I
    zr = mg.apply_block_preconditioner("rana_ld", A, dt, K, Acal @ x, mg.exact_block_solver(M, K, A, dt))
    assert np.linalg.norm(zr - x) < 1e-12 * np.linalg.norm(x)
    # the transpose of P_L (or P_LD) is the transposed operator itself: exact by backward substitution
    for kind in ("gs_lower", "rana_ld"):
        z2 = mg.apply_block_preconditioner(kind, A, dt, K, AcalT @ x, mg.exact_block_solver(M, K, A, dt),
                                           trans=True)
        assert np.linalg.norm(z2 - x) < 1e-12 * np.linalg.norm(x)


# ---------------------------------------------------------------- IA-form preconditioners


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("kind", ["jacobi", "gs_lower", "gs_upper", "rana_ld"])
def test_exact_ia_block_preconditioner_definition(kind, trans):
    # with exact blocks, P^{-1} v solves Atil^{-1} (x) M + dt I (x) K, and equals the AI-form
    # preconditioner applied to (Atil (x) I) v since P_IA = (Atil^{-1} (x) I) P_AI
    N, dt = 10, 1e-2
    kap = synth.grf_kappa(N, 4)
    M, K = fem.assemble(N, kap)
    A = T.radau_iia(3)["A"]
    L1, D, U1 = mg.ldu(A)
    Atil = {"jacobi": np.diag(np.diag(A)), "gs_lower": np.tril(A), "gs_upper": np.triu(A),
            "rana_ld": L1 @ np.diag(D)}[kind]
    n = (N - 1) ** 2
    v = np.random.default_rng(5).standard_normal(3 * n)
    z = mg.apply_ia_block_preconditioner(kind, A, dt, M, K, v, mg.exact_ia_block_solver(M, K, Atil, dt),
                                         trans=trans)
    P = step.coupled_matrix_ia(M, K, Atil, dt)
    if trans:
        P = P.T
    assert np.linalg.norm(P @ z - v) < 1e-12 * np.linalg.norm(v)
    At = Atil.T if trans else Atil
    mixed = (At @ v.reshape(3, -1)).ravel()
    z_ai = mg.apply_block_preconditioner(kind, A, dt, K, mixed, mg.exact_block_solver(M, K, Atil, dt),
                                         trans=trans)
    assert np.linalg.norm(z - z_ai) < 1e-12 * np.linalg.norm(z)


def test_ia_gs_lower_is_exact_for_dirk():
    N, dt = 10, 1e-2
    kap = synth.grf_kappa(N, 4)
    M, K = fem.assemble(N, kap)
    A = T.alexander()["A"]
    x = np.random.default_rng(6).standard_normal(3 * (N - 1) ** 2)
    v = step.coupled_matrix_ia(M, K, A, dt) @ x
    z = mg.apply_ia_block_preconditioner("gs_lower", A, dt, M, K, v, mg.exact_ia_block_solver(M, K, A, dt))
    assert np.linalg.norm(z - x) < 1e-12 * np.linalg.norm(x)


def test_vcycle_is_homogeneous_in_the_block():
    # one V-cycle on c M + dt a K: Jacobi-Chebyshev is invariant under scaling the operator and the coarse
    # solve scales with it, so V(B/c') = c' V(B); the IA block (1/a) M + dt K is (1/a)(M + dt a K)
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    hier = mg.Hierarchy(N, kap, dt, coarse_n=8)
    t = np.random.default_rng(10).standard_normal((N - 1) ** 2)
    for a in (0.2, 0.42):
        x1 = hier.vcycle(1.0, t, c=1.0 / a)
        x2 = a * hier.vcycle(a, t)
        assert np.linalg.norm(x1 - x2) < 1e-12 * np.linalg.norm(x2)
        # and it is not the identity map of the unscaled block (the scale matters)
        assert np.linalg.norm(hier.vcycle(a, t) - x1) > 0.1 * np.linalg.norm(x1)
