"""GPU parity of the multigrid kernels in the tile configurations the full-size workloads run, against the oracle's
CSR statement (oracle.mg, oracle.mmg), with the variable diffusivity of those workloads (kappa = exp(GRF seed 1)).

Levels with 512 or more elements per side run other kernel instantiations than the smaller grids of
test_gpu_mg.py / test_gpu_mmg.py: 64 x 16 tiles for the single-stage V-cycle (Section 3.1, the diagonal blocks
of eq:pcbjac / eq:pcbgs / eq:pcranald), 64 x 8 tiles for the monolithic cycle (Section 3.2, relaxation eq:Cinv),
and the block-triangular stage coupling fused into the finest DOWN kernel. FGMRES is flexible and checks its
true residual, so a mistake in these kernels would only show as more iterations in an end-to-end solve; here
they are compared node by node. 1024 - 1 interior nodes per side leave a ragged last tile in both directions.
"""
import numpy as np
import pytest

from oracle import fem, mg, mmg
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu

DT = 1e-3
TOL = {P.F64: 1e-12, P.F32: 2e-5, P.BF16: 3e-2}
_CACHE = {}


def _grid(N):
    """kappa, M, K and the single-stage oracle hierarchy at N (built once per session)."""
    if N not in _CACHE:
        kap = synth.grf_kappa(N, 1)
        M, K = fem.assemble(N, kap)
        _CACHE[N] = (kap, M, K, mg.Hierarchy(N, kap, DT))
    return _CACHE[N]


def _mmg_hier(N, splitting, transpose):
    key = ("mmg", N, splitting, transpose)
    if key not in _CACHE:
        kap = _grid(N)[0]
        A = OT.radau_iia(3)["A"]
        _CACHE[key] = mmg.MonolithicHierarchy(N, kap, DT, *mmg.mixing(A, splitting, transpose))
    return _CACHE[key]


@pytest.mark.parametrize("N", [512, 1024])
def test_vcycle_fullsize_fp64(N):
    kap, _, _, hier = _grid(N)
    A = OT.radau_iia(3)["A"]
    _, stp = make(N, kap, P.tableaux.radau_iia(3), DT)
    assert stp.levels == len(hier.sizes)
    for i in range(3):
        _, _, mus, _ = hier.block(A[i, i])
        for l in range(len(hier.sizes) - 1):
            assert abs(stp.mu(i, l) - mus[l]) <= 1e-11 * mus[l]
        t = synth.random_stage_block(N, 1, 30 + i).ravel()
        err = rel(host(stp.vcycle(i, dev(t))), hier.vcycle(A[i, i], t))
        print(f"N={N} stage {i} V-cycle FP64 rel err {err:.2e}")
        assert err < TOL[P.F64]


@pytest.mark.parametrize("prec", [P.F32, P.BF16])
def test_vcycle_fullsize_reduced_precision(prec):
    N = 1024
    kap, _, _, hier = _grid(N)
    A = OT.radau_iia(3)["A"]
    _, stp = make(N, kap, P.tableaux.radau_iia(3), DT, mg_precision=prec)
    for i in range(3):
        t = synth.random_stage_block(N, 1, 40 + i).ravel()
        err = rel(host(stp.vcycle(i, dev(t))), hier.vcycle(A[i, i], t))
        print(f"N={N} stage {i} V-cycle prec {prec} rel err {err:.2e}")
        assert err < TOL[prec]


# (preconditioner, splitting, transposed, precision): the headline path (P_L, AI, FP32 multigrid) and its FP64 and
# BF16 forms, the transposed system of the adjoint, Rana-LD in both splittings, P_U
_BLOCK_CASES = [
    ("gs_lower", "AI", False, P.F64), ("gs_lower", "AI", False, P.F32), ("gs_lower", "AI", False, P.BF16),
    ("gs_lower", "AI", True, P.F64), ("rana_ld", "AI", False, P.F64), ("rana_ld", "IA", False, P.F64),
    ("rana_ld", "IA", True, P.F32), ("gs_lower", "IA", False, P.F64), ("gs_upper", "AI", False, P.F64),
    ("jacobi", "AI", False, P.F32),
]
_PC = {"jacobi": P.PC_JACOBI, "gs_lower": P.PC_GS_LOWER, "gs_upper": P.PC_GS_UPPER, "rana_ld": P.PC_RANA_LD}


@pytest.mark.parametrize("kind,splitting,transpose,prec", _BLOCK_CASES)
def test_block_preconditioner_fullsize(kind, splitting, transpose, prec):
    N = 1024
    kap, M, K, hier = _grid(N)
    A = OT.radau_iia(3)["A"]
    Atil = mg.preconditioner_matrix(kind, A)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), DT, precond=_PC[kind], mg_precision=prec,
                  splitting=P.SPLIT_AI if splitting == "AI" else P.SPLIT_IA)
    v = synth.random_stage_block(N, 3, 50).ravel()
    z = host(stp.apply_preconditioner(dev(v), transpose=transpose))
    if splitting == "AI":
        ref = mg.apply_block_preconditioner(kind, A, DT, K, v, mg.vcycle_block_solver(hier, Atil), trans=transpose)
    else:
        ref = mg.apply_ia_block_preconditioner(kind, A, DT, M, K, v, mg.vcycle_ia_block_solver(hier, Atil),
                                               trans=transpose)
    err = rel(z, ref)
    print(f"N={N} {kind} {splitting} trans={transpose} prec {prec} rel err {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("N,splitting,transpose,prec", [(512, "AI", False, P.F64), (512, "AI", True, P.F64),
                                                        (512, "IA", False, P.F64), (512, "AI", False, P.BF16),
                                                        (1024, "AI", False, P.F64), (1024, "AI", False, P.F32)])
def test_mmg_vcycle_fullsize(N, splitting, transpose, prec):
    kap = _grid(N)[0]
    H = _mmg_hier(N, splitting, transpose)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), DT, precond=P.PC_MONOLITHIC, mg_precision=prec,
                  splitting=P.SPLIT_AI if splitting == "AI" else P.SPLIT_IA)
    assert stp.mmg_levels == len(H.sizes)
    if prec == P.F64:
        for l in range(len(H.sizes) - 1):
            assert abs(stp.mmg_mu(l, transpose) - H.mus[l]) <= 1e-11 * H.mus[l]
    v = synth.random_stage_block(N, 3, 60).ravel()
    err = rel(host(stp.apply_preconditioner(dev(v), transpose=transpose)), H.vcycle(v))
    print(f"N={N} monolithic {splitting} trans={transpose} prec {prec} rel err {err:.2e}")
    assert err < TOL[prec]
