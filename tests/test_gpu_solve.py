"""GPU parity: FGMRES stage solve (a5), time stepping (a1+a5+a6) and the mixed-precision form (a7)
against the oracle's exact direct solves and closed forms."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, step
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu


def _max_rel(gpu_list, ora_list):
    return max(rel(a, b) for a, b in zip(gpu_list, ora_list))


@pytest.mark.parametrize("pc", [P.PC_JACOBI, P.PC_GS_LOWER, P.PC_GS_UPPER, P.PC_RANA_LD])
@pytest.mark.parametrize("transpose", [False, True])
def test_solve_stages_matches_direct(pc, transpose):
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    otab = OT.radau_iia(3)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, precond=pc, rtol=1e-12)
    f = synth.random_stage_block(N, 3, 21).ravel()
    k, stats = stp.solve_stages(dev(f), transpose=transpose)
    ref = step.CoupledLU(M, K, otab["A"], dt).solve(f, trans=transpose)
    Acal = step.coupled_matrix(M, K, otab["A"].T if transpose else otab["A"], dt)
    assert np.linalg.norm(Acal @ host(k) - f) <= 1.01e-12 * np.linalg.norm(f)
    assert stats["last_rel_resid"] <= 1e-12
    assert rel(host(k), ref) < 1e-9
    assert stats["fgmres_its_total"] > 1


@pytest.mark.parametrize("pc", [P.PC_JACOBI, P.PC_GS_LOWER, P.PC_GS_UPPER, P.PC_RANA_LD])
@pytest.mark.parametrize("transpose", [False, True])
def test_ia_solve_stages_matches_direct(pc, transpose):
    # eq:block_struct_IA: (A^{-1} (x) M + dt I (x) K) w = f, or its transpose
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    otab = OT.radau_iia(3)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, precond=pc, rtol=1e-12, splitting=P.SPLIT_IA)
    f = synth.random_stage_block(N, 3, 22).ravel()
    w, stats = stp.solve_stages(dev(f), transpose=transpose)
    Acal = step.coupled_matrix_ia(M, K, otab["A"], dt)
    if transpose:
        Acal = Acal.T.tocsc()
    ref = spla.spsolve(Acal, f)
    y = host(stp.apply_stage_operator(dev(ref), transpose=transpose))
    assert rel(y, Acal @ ref) < 1e-14
    assert np.linalg.norm(Acal @ host(w) - f) <= 1.01e-12 * np.linalg.norm(f)
    assert stats["last_rel_resid"] <= 1e-12
    assert rel(host(w), ref) < 1e-9


@pytest.mark.parametrize("tname,pc,prec,tol", [("gl4", P.PC_GS_LOWER, P.F64, 1e-10), ("gl4", P.PC_RANA_LD, P.F64, 1e-10),
                                               ("radau3", P.PC_RANA_LD, P.F32, 1e-8),
                                               ("lobatto", P.PC_GS_LOWER, P.F64, 1e-10),
                                               ("alexander", P.PC_GS_LOWER, P.F64, 1e-10)])
def test_ia_advance_matches_oracle(tname, pc, prec, tol):
    # the IA form integrates the same step: compare with the oracle's IA run (and so with the AI one)
    N, dt, nsteps = 128, 5e-4, 4
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    otab = {"gl4": OT.gauss_legendre(4), "radau3": OT.radau_iia(3), "lobatto": OT.lobatto_iiic2(),
            "alexander": OT.alexander()}[tname]
    ptab = {"gl4": P.tableaux.gauss_legendre(4), "radau3": P.tableaux.radau_iia(3),
            "lobatto": P.tableaux.lobatto_iiic2(), "alexander": P.tableaux.alexander()}[tname]
    _, stp = make(N, kap, ptab, dt, precond=pc, rtol=1e-12, splitting=P.SPLIT_IA, mg_precision=prec)
    u = dev(u0)
    gpu = []
    for _ in range(nsteps):
        stp.advance(u, 1)
        gpu.append(host(u))
    ora = step.run(N, kap, otab, dt, nsteps, u0, splitting="IA")[1:]
    assert _max_rel(gpu, ora) < tol


def test_ia_rejects_singular_tableau():
    N = 16
    prob = P.Problem(N, dev(np.ones(N * N)))
    tab = {"A": np.array([[0.5, 0.5], [0.5, 0.5]]), "b": np.array([0.5, 0.5]), "c": np.array([1.0, 1.0])}
    P.Stepper(prob, tab, 1e-3, precond=P.PC_JACOBI)  # the AI form only needs a_ii > 0
    with pytest.raises(P.IrkError) as e:
        P.Stepper(prob, tab, 1e-3, precond=P.PC_JACOBI, splitting=P.SPLIT_IA)
    assert e.value.code == P.IRK_EINVAL


def test_config1_decay():
    # 32x32, Radau IIA(2), dt = 1/32, 10 steps, u0 = sin(pi x) sin(pi y)
    N, dt = 32, 1.0 / 32
    u0 = synth.sine_mode_vector(N, 1, 1)
    _, stp = make(N, np.ones(N * N), P.tableaux.radau_iia(2), dt, rtol=1e-13)
    u = dev(u0)
    gpu = [u0.copy()]
    for _ in range(10):
        stp.advance(u, 1)
        gpu.append(host(u))
    ora = step.run(N, None, OT.radau_iia(2), dt, 10, u0)
    lam = step.discrete_eigenvalue(N, 1, 1)
    R = OT.stability_function(OT.radau_iia(2), -dt * lam)[0].real
    assert _max_rel(gpu, ora) < 1e-10
    assert rel(gpu[-1], R**10 * u0) < 1e-10


@pytest.mark.parametrize("N", [64, 128])
def test_config2_shape_closed_form(N):
    # Radau IIA(3), dt = 1e-3, 16 seeded sine modes, kappa = 1, P_L + FP64 V-cycle: closed form R(-dt lam)^n
    dt, nsteps = 1e-3, 10
    u0, amps = synth.sine_modes_u0(N, 0)
    _, stp = make(N, np.ones(N * N), P.tableaux.radau_iia(3), dt, rtol=1e-12)
    u = dev(u0)
    gpu = []
    for _ in range(nsteps):
        _, st = stp.advance(u, 1)
        gpu.append(host(u))
    cf = step.closed_form_modes(N, OT.radau_iia(3), dt, nsteps, amps)[1:]
    assert _max_rel(gpu, cf) < 1e-10


@pytest.mark.parametrize("pc", [P.PC_JACOBI, P.PC_GS_LOWER, P.PC_RANA_LD])
def test_config3_shape_gl4(pc):
    # variable kappa (GRF), Gauss-Legendre(4), dt = 5e-4; direct coupled oracle
    N, dt, nsteps = 128, 5e-4, 4
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    _, stp = make(N, kap, P.tableaux.gauss_legendre(4), dt, precond=pc, rtol=1e-12)
    u = dev(u0)
    gpu = []
    its = 0
    for _ in range(nsteps):
        _, st = stp.advance(u, 1)
        its += st["fgmres_its_total"]
        gpu.append(host(u))
    ora = step.run(N, kap, OT.gauss_legendre(4), dt, nsteps, u0)[1:]
    assert _max_rel(gpu, ora) < 1e-10


@pytest.mark.parametrize("prec,tol", [(P.F64, 1e-10), (P.F32, 1e-8), (P.BF16, 1e-8)])
def test_config4_shape_mixed_precision(prec, tol):
    # Radau IIA(3), dt = 1e-3, GRF kappa; multigrid in FP64 / FP32 / BF16 storage, outer FGMRES FP64 at rtol 1e-10
    N, dt, nsteps = 128, 1e-3, 5
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, mg_precision=prec, rtol=1e-10)
    u = dev(u0)
    gpu = []
    for _ in range(nsteps):
        stp.advance(u, 1)
        gpu.append(host(u))
    ora = step.run(N, kap, OT.radau_iia(3), dt, nsteps, u0)[1:]
    assert _max_rel(gpu, ora) < tol


def test_selective_reorthogonalisation_and_prev_guess():
    N, dt, nsteps = 64, 1e-3, 4
    kap = synth.grf_kappa(N, 2)
    u0, _ = synth.sine_modes_u0(N, 0)
    ora = step.run(N, kap, OT.radau_iia(3), dt, nsteps, u0)[-1]
    for opts in ({"orth": P.ORTH_CGS_SELECTIVE}, {"initial_guess": P.GUESS_PREV}):
        _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-12, **opts)
        u = dev(u0)
        stp.advance(u, nsteps)
        assert rel(host(u), ora) < 1e-10


def test_dirk_gs_lower_with_exact_blocks_converges_in_one_iteration():
    # lower-triangular A: P_L equals the stage operator; with one level the V-cycle is an exact solve, so
    # one Arnoldi step solves the system. With CGS2 the residual estimate shows it at once; DCGS2 predicts
    # the next direction's norm by subtraction (|w|^2 - |h|^2, exact only down to sqrt(eps)|w|) and sees it
    # one step later, when that direction is re-orthogonalised and measured.
    N, dt = 8, 1e-2
    kap = synth.grf_kappa(N, 3)
    f = synth.random_stage_block(N, 3, 2).ravel()
    sols = {}
    for orth, its in ((P.ORTH_CGS2, 1), (P.ORTH_DCGS2, 2)):
        _, stp = make(N, kap, P.tableaux.alexander(), dt, precond=P.PC_GS_LOWER, rtol=1e-12, orth=orth)
        assert stp.levels == 1
        k, stats = stp.solve_stages(dev(f))
        assert 1 <= stats["fgmres_its_total"] <= its
        # the transposed system is preconditioned by the transpose of P_L, exact here as well
        kt, stats = stp.solve_stages(dev(f), transpose=True)
        assert 1 <= stats["fgmres_its_total"] <= its
        sols[orth] = (host(k), host(kt))
        # s = 1 (backward Euler) with P_D likewise
        _, stp1 = make(N, kap, P.tableaux.radau_iia(1), dt, precond=P.PC_JACOBI, rtol=1e-12, orth=orth)
        _, stats = stp1.solve_stages(dev(f[: (N - 1) ** 2]))
        assert 1 <= stats["fgmres_its_total"] <= its
    # whatever step notices it, both processes return the exact solve (forward and transposed)
    for a, b in zip(sols[P.ORTH_CGS2], sols[P.ORTH_DCGS2]):
        assert rel(b, a) < 1e-11


def test_iterations_grow_with_stages_and_gs_beats_jacobi():
    # paper's trend (Section 4.1 heat study): P_D and P_L iteration counts grow with s; P_L needs fewer than P_D
    N, dt = 128, 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    its = {}
    for pc in (P.PC_JACOBI, P.PC_GS_LOWER):
        for s in (1, 2, 3):
            _, stp = make(N, kap, P.tableaux.radau_iia(s), dt, precond=pc, rtol=1e-10)
            u = dev(u0)
            _, st = stp.advance(u, 2)
            its[(pc, s)] = st["fgmres_its_total"] / 2
    assert its[(P.PC_JACOBI, 3)] > its[(P.PC_JACOBI, 1)]
    assert its[(P.PC_GS_LOWER, 3)] > its[(P.PC_GS_LOWER, 1)]
    assert its[(P.PC_GS_LOWER, 3)] < its[(P.PC_JACOBI, 3)]


def test_rana_ld_iterations_flat_in_stages():
    # paper's trend (Section 4.1 heat study): P_LD iteration counts stay nearly flat over the number of
    # stages while P_L's grow; P_LD needs no more iterations than P_L
    N, dt = 128, 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    its = {}
    for pc in (P.PC_GS_LOWER, P.PC_RANA_LD):
        for s in (1, 2, 3, 4):
            _, stp = make(N, kap, P.tableaux.radau_iia(s), dt, precond=pc, rtol=1e-10)
            u = dev(u0)
            _, st = stp.advance(u, 2)
            its[(pc, s)] = st["fgmres_its_total"] / 2
    print(its)
    for s in (2, 3, 4):
        assert its[(P.PC_RANA_LD, s)] <= its[(P.PC_GS_LOWER, s)]
    assert its[(P.PC_RANA_LD, 1)] == its[(P.PC_GS_LOWER, 1)]
    assert its[(P.PC_RANA_LD, 4)] - its[(P.PC_RANA_LD, 1)] < its[(P.PC_GS_LOWER, 4)] - its[(P.PC_GS_LOWER, 1)]


def test_rana_ld_rejects_nonpositive_pivot():
    # A = [[1, 2], [2, 1]] has a_ii > 0 but the second LDU pivot is 1 - 4 = -3
    N = 16
    prob = P.Problem(N, dev(np.ones(N * N)))
    tab = {"A": np.array([[1.0, 2.0], [2.0, 1.0]]), "b": np.array([0.5, 0.5]), "c": np.array([3.0, 3.0])}
    with pytest.raises(P.IrkError) as e:
        P.Stepper(prob, tab, 1e-3, precond=P.PC_RANA_LD)
    assert e.value.code == P.IRK_EINVAL


def test_enoconv_keeps_last_good_state():
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-14, max_it=1)
    u = dev(u0)
    rc, st = stp.advance(u, 3, check=False)
    assert rc == P.IRK_ENOCONV
    assert st["failed_step"] == 0 and st["steps_done"] == 0
    assert np.array_equal(host(u), u0)


@pytest.mark.parametrize("orth,pc", [(P.ORTH_DCGS2, P.PC_GS_LOWER), (P.ORTH_CGS2, P.PC_GS_LOWER),
                                     (P.ORTH_DCGS2, P.PC_MONOLITHIC)])
def test_ebreakdown_on_non_finite_data(orth, pc):
    # a NaN in the stage right-hand side and an infinity in the state are reported as IRK_EBREAKDOWN (the Arnoldi
    # steps queued ahead of the host's norm check compute on the non-finite values, and the flat vector kernels
    # then write non-finite values into the boundary ring of the work planes); the stepper clears its work planes
    # and stays usable: its next solves give the same bits as a new stepper's
    N, dt = 32, 1e-3
    kap = synth.grf_kappa(N, 1)
    tab = P.tableaux.radau_iia(3)
    _, stp = make(N, kap, tab, dt, rtol=1e-12, orth=orth, precond=pc)
    f = synth.random_stage_block(N, 3, 4).ravel()
    bad = f.copy()
    bad[17] = np.nan
    with pytest.raises(P.IrkError) as e:
        stp.solve_stages(dev(bad))
    assert e.value.code == P.IRK_EBREAKDOWN
    u0, _ = synth.sine_modes_u0(N, 0)
    ub = u0.copy()
    ub[5] = np.inf
    rc, st = stp.advance(dev(ub), 2, check=False)
    assert rc == P.IRK_EBREAKDOWN and st["failed_step"] == 0 and st["steps_done"] == 0
    x, _ = stp.solve_stages(dev(f))
    _, fresh = make(N, kap, tab, dt, rtol=1e-12, orth=orth, precond=pc)
    x2, _ = fresh.solve_stages(dev(f))
    assert np.array_equal(host(x), host(x2))
    u, u2 = dev(u0), dev(u0)
    stp.advance(u, 2)
    fresh.advance(u2, 2)
    assert np.array_equal(host(u), host(u2))


def test_invalid_kappa_rejected():
    N = 16
    kap = np.ones(N * N)
    kap[5] = np.nan
    with pytest.raises(P.IrkError) as e:
        P.Problem(N, dev(kap))
    assert e.value.code == P.IRK_EINVAL
    kap[5] = -1.0
    with pytest.raises(P.IrkError):
        P.Problem(N, dev(kap))


def test_invalid_tableau_rejected():
    N = 16
    prob = P.Problem(N, dev(np.ones(N * N)))
    explicit = {"A": np.array([[0.0, 0.0], [1.0, 0.0]]), "b": np.array([0.5, 0.5]), "c": np.array([0.0, 1.0])}
    with pytest.raises(P.IrkError) as e:
        P.Stepper(prob, explicit, 1e-3)
    assert e.value.code == P.IRK_EINVAL


@pytest.mark.parametrize("prec", [P.F64, P.F32])
def test_graph_replay_matches_eager_bitwise(prec):
    # every Arnoldi step is replayed from a captured graph; eager launches must give identical bits
    N, dt, nsteps = 64, 1e-3, 3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    outs = []
    for g in (0, 1):
        _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, use_graphs=g, mg_precision=prec, restart=6)
        u = dev(u0)
        stp.advance(u, nsteps)  # restart = 6 forces restarts: graphs replay across cycles and steps
        u2 = dev(u0)
        stp.advance(u2, nsteps)  # second call: replays again after eager pack/unpack work
        outs.append((host(u), host(u2)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[1][0], outs[1][1])


# ---------------------------------------------------------------- DIRK stage type (Section 2.3)

_DIRK = {"alexander": (OT.alexander, P.tableaux.alexander), "wso433": (OT.wsodirk433, P.tableaux.wsodirk433)}


@pytest.mark.parametrize("tname", ["alexander", "wso433"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("N", [64, 128])
def test_dirk_solve_stages_matches_direct(tname, transpose, N):
    # N = 128 has three multigrid levels: the coarse-level power iterations share the stage right-hand side's
    # scratch buffer, whose fine-layout boundary and padding must be zero again afterwards
    dt = 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    otab, ptab = _DIRK[tname][0](), _DIRK[tname][1]()
    s = otab["A"].shape[0]
    _, stp = make(N, kap, ptab, dt, rtol=1e-12, stage_type=P.STAGE_DIRK)
    f = synth.random_stage_block(N, s, 23).ravel()
    k, stats = stp.solve_stages(dev(f), transpose=transpose)
    # exact stage-by-stage solves of the oracle's DIRK tier (equal to the coupled LU, pinned on the CPU)
    ref = step.dirk_solve(M, K, otab["A"], dt, f, trans=transpose)
    assert stats["solves"] == s and stats["fgmres_its_total"] >= s
    assert rel(host(k), ref) < 1e-10


@pytest.mark.parametrize("tname,prec,tol", [("alexander", P.F64, 1e-10), ("wso433", P.F64, 1e-10),
                                            ("wso433", P.F32, 1e-8)])
def test_dirk_advance_matches_oracle(tname, prec, tol):
    N, dt, nsteps = 128, 1e-3, 4
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    otab, ptab = _DIRK[tname][0](), _DIRK[tname][1]()
    _, stp = make(N, kap, ptab, dt, rtol=1e-12, stage_type=P.STAGE_DIRK, mg_precision=prec)
    u = dev(u0)
    gpu = []
    for _ in range(nsteps):
        stp.advance(u, 1)
        gpu.append(host(u))
    ora = step.run(N, kap, otab, dt, nsteps, u0, tier="dirk")[1:]
    assert _max_rel(gpu, ora) < tol


def test_dirk_closed_form_and_coupled_agree():
    # kappa = 1: u_n = sum alpha R(-dt lam)^n phi with the DIRK's stability function; the coupled solve of
    # the same tableau (P_L, exact up to the V-cycles) gives the same steps
    N, dt, nsteps = 64, 2e-3, 5
    u0, amps = synth.sine_modes_u0(N, 0)
    kap = np.ones(N * N)
    cf = step.closed_form_modes(N, OT.alexander(), dt, nsteps, amps)
    outs = {}
    for st_type in (P.STAGE_DIRK, P.STAGE_COUPLED):
        _, stp = make(N, kap, P.tableaux.alexander(), dt, rtol=1e-12, stage_type=st_type)
        u = dev(u0)
        stp.advance(u, nsteps)
        outs[st_type] = host(u)
        assert rel(outs[st_type], cf[nsteps]) < 1e-10
    assert rel(outs[P.STAGE_DIRK], outs[P.STAGE_COUPLED]) < 1e-10


def test_dirk_rejects_full_tableau_and_ia():
    N = 16
    prob = P.Problem(N, dev(np.ones(N * N)))
    for tab, opts in ((P.tableaux.radau_iia(3), {}), (P.tableaux.alexander(), {"splitting": P.SPLIT_IA})):
        with pytest.raises(P.IrkError) as e:
            P.Stepper(prob, tab, 1e-3, stage_type=P.STAGE_DIRK, **opts)
        assert e.value.code == P.IRK_EINVAL


# ---------------------------------------------------------------- delayed CGS2 Arnoldi process


@pytest.mark.parametrize("pc,splitting,restart", [(P.PC_GS_LOWER, P.SPLIT_AI, 30), (P.PC_MONOLITHIC, P.SPLIT_AI, 30),
                                                  (P.PC_RANA_LD, P.SPLIT_IA, 30), (P.PC_GS_LOWER, P.SPLIT_AI, 3)])
@pytest.mark.parametrize("transpose", [False, True])
def test_dcgs2_solve_stages_matches_direct(pc, splitting, restart, transpose):
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    A = OT.radau_iia(3)["A"]
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, precond=pc, splitting=splitting, rtol=1e-12,
                  orth=P.ORTH_DCGS2, restart=restart)
    f = synth.random_stage_block(N, 3, 25).ravel()
    x, stats = stp.solve_stages(dev(f), transpose=transpose)
    Acal = step.coupled_matrix(M, K, A, dt) if splitting == P.SPLIT_AI else step.coupled_matrix_ia(M, K, A, dt)
    if transpose:
        Acal = Acal.T.tocsc()
    ref = spla.spsolve(Acal, f)
    assert np.linalg.norm(Acal @ host(x) - f) <= 1.01e-12 * np.linalg.norm(f)
    assert rel(host(x), ref) < 1e-9
    if restart == 3:
        assert stats["restarts_total"] >= 1


def test_dcgs2_iterations_match_cgs2():
    # the delayed form builds the same Krylov space: the iteration counts agree with CGS2 (up to one)
    N, dt = 128, 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    its, us = {}, {}
    for orth in (P.ORTH_CGS2, P.ORTH_DCGS2):
        _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-10, orth=orth)
        u = dev(u0)
        _, st = stp.advance(u, 3)
        its[orth] = st["fgmres_its_total"]
        us[orth] = host(u)
    assert abs(its[P.ORTH_DCGS2] - its[P.ORTH_CGS2]) <= 3
    assert rel(us[P.ORTH_DCGS2], us[P.ORTH_CGS2]) < 1e-9


@pytest.mark.parametrize("prec", [P.F64, P.F32])
def test_dcgs2_graph_replay_matches_eager_bitwise(prec):
    N, dt, nsteps = 64, 1e-3, 3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    outs = []
    for g in (0, 1):
        _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, use_graphs=g, mg_precision=prec, restart=6,
                      orth=P.ORTH_DCGS2)
        u = dev(u0)
        stp.advance(u, nsteps)
        u2 = dev(u0)
        stp.advance(u2, nsteps)
        outs.append((host(u), host(u2)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[1][0], outs[1][1])


@pytest.mark.parametrize("pc,prec", [(P.PC_GS_LOWER, P.F32), (P.PC_MONOLITHIC, P.F32), (P.PC_JACOBI, P.F64)])
def test_lookahead_modes_agree_bitwise(pc, prec):
    # a step queued ahead of the convergence test and then not used writes only Krylov vectors beyond the
    # ones the solution is built from, so every mode gives the same bits; ALWAYS discards one at the end of
    # each solve (unless it ends at a restart boundary), OFF never
    N, dt = 96, 1e-3
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    otab = OT.radau_iia(3)
    f = synth.random_stage_block(N, 3, 29).ravel()
    out = {}
    for look in (P.LOOKAHEAD_OFF, P.LOOKAHEAD_ADAPTIVE, P.LOOKAHEAD_ALWAYS):
        _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, precond=pc, mg_precision=prec, rtol=1e-10,
                      lookahead=look)
        k, stats = stp.solve_stages(dev(f))
        out[look] = (host(k), stats)
    k0, s0 = out[P.LOOKAHEAD_OFF]
    for look in (P.LOOKAHEAD_ADAPTIVE, P.LOOKAHEAD_ALWAYS):
        assert np.array_equal(out[look][0], k0)
        assert out[look][1]["fgmres_its_total"] == s0["fgmres_its_total"]
    assert s0["arnoldi_discarded"] == 0
    assert out[P.LOOKAHEAD_ALWAYS][1]["arnoldi_discarded"] >= 1
    ref = step.CoupledLU(M, K, otab["A"], dt).solve(f)
    assert rel(k0, ref) < 1e-8


def test_lookahead_always_matches_off_over_dirk_steps():
    # several single-stage solves per step, each ending with a discarded step under ALWAYS
    N, dt, nsteps = 96, 1e-3, 3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    res = []
    for look in (P.LOOKAHEAD_OFF, P.LOOKAHEAD_ALWAYS):
        _, stp = make(N, kap, _DIRK["wso433"][1](), dt, rtol=1e-12, stage_type=P.STAGE_DIRK, lookahead=look)
        u = dev(u0)
        _, stats = stp.advance(u, nsteps)
        res.append((host(u), stats))
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1]["arnoldi_discarded"] == 0 and res[1][1]["arnoldi_discarded"] >= nsteps


def test_lookahead_rejects_unknown_mode():
    kap = synth.grf_kappa(16, 1)
    with pytest.raises(P.IrkError):
        make(16, kap, P.tableaux.radau_iia(2), 1e-3, lookahead=3)


@pytest.mark.parametrize("N,prec,pc,split,orth,stage", [
    (128, P.F32, P.PC_GS_LOWER, P.SPLIT_AI, P.ORTH_DCGS2, P.STAGE_COUPLED),
    (128, P.BF16, P.PC_RANA_LD, P.SPLIT_IA, P.ORTH_DCGS2, P.STAGE_COUPLED),
    (128, P.F32, P.PC_MONOLITHIC, P.SPLIT_AI, P.ORTH_CGS2, P.STAGE_COUPLED),
    (128, P.F32, P.PC_GS_LOWER, P.SPLIT_AI, P.ORTH_DCGS2, P.STAGE_DIRK),
    (33, P.F32, P.PC_GS_UPPER, P.SPLIT_AI, P.ORTH_DCGS2, P.STAGE_COUPLED),
    (512, P.F32, P.PC_GS_LOWER, P.SPLIT_AI, P.ORTH_DCGS2, P.STAGE_COUPLED)])
def test_fp32_flexible_basis_gives_the_fp64_basis_bits(N, prec, pc, split, orth, stage):
    # the mixed form keeps the preconditioned vectors Z_j in FP32; the FP32 multigrid computed them, so the
    # stored values are those an FP64 basis holds: steps, transposed stage solves and the adjoint agree bit for bit
    kap = synth.grf_kappa(N, 1)
    tab = P.tableaux.alexander() if stage == P.STAGE_DIRK else P.tableaux.radau_iia(3)
    opts = dict(mg_precision=prec, precond=pc, splitting=split, orth=orth, stage_type=stage, rtol=1e-10)
    res = []
    for basis_f64 in (0, 1):
        _, stp = make(N, kap, tab, 1e-3, basis_f64=basis_f64, **opts)
        u = dev(synth.sine_modes_u0(N, 0)[0])
        _, st = stp.advance(u, 3)
        k, stt = stp.solve_stages(dev(synth.random_stage_block(N, 3, 4).ravel()), transpose=True)
        out = [host(u), host(k), st["fgmres_its_total"], stt["fgmres_its_total"]]
        if N == 128 and pc == P.PC_GS_LOWER and stage == P.STAGE_COUPLED:
            lam0, grad, _ = stp.adjoint(dev(synth.sine_modes_u0(N, 0)[0]), 4, 2, dev(synth.sine_modes_u0(N, 1)[0]))
            out += [host(lam0), host(grad)]
        res.append(out)
    for a, b in zip(*res):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    with pytest.raises(P.IrkError):
        make(16, synth.grf_kappa(16, 1), P.tableaux.radau_iia(3), 1e-3, basis_f64=2)
