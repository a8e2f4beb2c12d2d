"""Pins for oracle.mmg: reduction to the single-stage cycle, the additive Schwarz definition, exactness,
contraction and the eigenvalue estimate."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, mg, mmg, step
from oracle import tableaux as T
import synth


def test_one_stage_is_the_single_stage_cycle():
    # s = 1, A = [[a]]: the monolithic cycle is the single-stage V-cycle for M + dt a K (written separately)
    N, dt, a = 64, 1e-3, 0.3
    kap = synth.grf_kappa(N, 1)
    Cm, Ck = mmg.mixing(np.array([[a]]))
    H = mmg.MonolithicHierarchy(N, kap, dt, Cm, Ck, coarse_n=8)
    h = mg.Hierarchy(N, kap, dt, coarse_n=8)
    assert H.sizes == h.sizes
    t = np.random.default_rng(1).standard_normal((N - 1) ** 2)
    ref = h.vcycle(a, t)
    assert np.linalg.norm(H.vcycle(t) - ref) < 1e-12 * np.linalg.norm(ref)
    assert abs(H.mus[0] - h.block(a)[2][0]) < 1e-12 * H.mus[0]


@pytest.mark.parametrize("splitting,trans", [("AI", False), ("IA", False), ("AI", True)])
def test_additive_schwarz_definition(splitting, trans):
    # eq:Cinv written out on a tiny grid: A_v = p_v^T Acal p_v from the assembled coupled operator, summed
    N, dt = 5, 0.05
    kap = synth.grf_kappa(N, 2)
    M, K = fem.assemble(N, kap)
    A = T.radau_iia(3)["A"]
    Cm, Ck = mmg.mixing(A, splitting, trans)
    Acal = mmg.coupled_level_matrix(M, K, Cm, Ck, dt).toarray()
    ref_op = (step.coupled_matrix(M, K, A.T if trans else A, dt) if splitting == "AI" else
              step.coupled_matrix_ia(M, K, A.T if trans else A, dt)).toarray()
    assert np.abs(Acal - ref_op).max() < 1e-14 * np.abs(ref_op).max()
    n, s = (N - 1) ** 2, 3
    Cinv = np.zeros((s * n, s * n))
    for v in range(n):
        p = np.zeros((s * n, s))
        for q in range(s):
            p[q * n + v, q] = 1.0
        Cinv += p @ np.linalg.inv(p.T @ Acal @ p) @ p.T
    r = np.random.default_rng(2).standard_normal(s * n)
    blocks = mmg.patch_blocks(M, K, Cm, Ck, dt)
    assert np.linalg.norm(mmg.additive_schwarz(blocks, r) - Cinv @ r) < 1e-13 * np.linalg.norm(Cinv @ r)
    x = np.random.default_rng(3).standard_normal(s * n)
    assert abs(mmg.patch_energy(blocks, x) - x @ np.linalg.solve(Cinv, x)) < 1e-10 * abs(mmg.patch_energy(blocks, x))


def test_single_level_is_an_exact_solve():
    N, dt = 16, 1e-2
    kap = synth.grf_kappa(N, 3)
    A = T.gauss_legendre(4)["A"]
    H = mmg.MonolithicHierarchy(N, kap, dt, *mmg.mixing(A), coarse_n=16, max_coarse=4 * 15 * 15)
    assert H.sizes == [16]
    M, K = fem.assemble(N, kap)
    t = np.random.default_rng(4).standard_normal(4 * 15 * 15)
    x = H.vcycle(t)
    assert np.linalg.norm(step.coupled_matrix(M, K, A, dt) @ x - t) < 1e-12 * np.linalg.norm(t)


def test_level_rule():
    assert mmg.level_sizes(1024, 3) == [1024, 512, 256, 128, 64, 32, 16]
    assert mmg.level_sizes(1024, 1) == [1024, 512, 256, 128, 64, 32]
    assert mmg.level_sizes(1024, 8) == [1024, 512, 256, 128, 64, 32, 16, 8]
    assert mmg.level_sizes(96, 3) == [96, 48, 24, 12]  # 3 * 23^2 > 1024
    assert mmg.level_sizes(66, 3) == [66, 33]


@pytest.mark.parametrize("splitting", ["AI", "IA"])
def test_vcycle_contracts(splitting):
    # as a stationary iteration the monolithic V-cycle reduces the error of the coupled system every cycle
    N, dt = 64, 1e-3
    kap = synth.grf_kappa(N, 1)
    A = T.radau_iia(3)["A"]
    H = mmg.MonolithicHierarchy(N, kap, dt, *mmg.mixing(A, splitting))
    Acal = H.ops[0]
    e = np.random.default_rng(5).standard_normal(Acal.shape[0])
    for _ in range(3):
        e2 = e - H.vcycle(Acal @ e)
        assert np.linalg.norm(e2) < 0.3 * np.linalg.norm(e)
        e = e2


def test_power_estimate_near_the_extreme_eigenvalue():
    # the quotient after power iteration lands near the largest real part of the spectrum of C^{-1} Acal
    N, dt = 8, 5e-2
    kap = synth.grf_kappa(N, 1)
    A = T.radau_iia(3)["A"]
    H = mmg.MonolithicHierarchy(N, kap, dt, *mmg.mixing(A), coarse_n=2, max_coarse=1, power_its=60)
    blk = H.blocks[0]
    n = H.ops[0].shape[0]
    CA = np.column_stack([mmg.additive_schwarz(blk, H.ops[0] @ np.eye(n)[:, i]) for i in range(n)])
    lam = np.linalg.eigvals(CA)
    assert np.all(lam.real > 0)
    assert 0.8 * lam.real.max() < H.mus[0] < 1.2 * np.abs(lam).max()
