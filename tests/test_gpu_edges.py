"""GPU edge cases: the largest grids in the suite (closed form), the smallest grid, ragged grids whose level sizes
fit no tile, the largest stage count, empty work, non-finite data and a device allocation that cannot succeed."""
import numpy as np
import pytest

from oracle import fem, step
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,pc", [(2048, P.PC_GS_LOWER), (2048, P.PC_MONOLITHIC), (4096, P.PC_GS_LOWER)])
def test_largest_grid_closed_form(N, pc):
    # 2048^2 (4.2M interior nodes, 12.6M stage unknowns) and 4096^2 (16.8M nodes, 50.3M stage unknowns, ten
    # multigrid levels), kappa = 1: sine modes decay by R(-dt lam) exactly
    dt, nsteps = 1e-3, 2
    u0, amps = synth.sine_modes_u0(N, 0)
    _, stp = make(N, np.ones(N * N), P.tableaux.radau_iia(3), dt, rtol=1e-10, precond=pc, mg_precision=P.F32)
    cf = step.closed_form_modes(N, OT.radau_iia(3), dt, nsteps, amps)
    u = dev(u0)
    for k in range(1, nsteps + 1):
        stp.advance(u, 1)
        assert rel(host(u), cf[k]) < 1e-8


@pytest.mark.parametrize("pc", [P.PC_GS_LOWER, P.PC_MONOLITHIC])
def test_smallest_grid(pc):
    # N = 2: one interior node; every multigrid path reduces to the dense coarsest solve
    N, dt = 2, 0.1
    kap = np.array([1.0, 2.0, 3.0, 4.0])
    u0 = np.array([1.0])
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt, rtol=1e-13, precond=pc)
    u = dev(u0)
    stp.advance(u, 3)
    ref = step.run(N, kap, OT.radau_iia(3), dt, 3, u0, tier="dense")[-1]
    assert rel(host(u), ref) < 1e-12


@pytest.mark.parametrize("name,pc,split,stage", [("radau3", P.PC_GS_LOWER, P.SPLIT_AI, P.STAGE_COUPLED),
                                                 ("radau3", P.PC_RANA_LD, P.SPLIT_IA, P.STAGE_COUPLED),
                                                 ("radau3", P.PC_MONOLITHIC, P.SPLIT_AI, P.STAGE_COUPLED),
                                                 ("alexander", P.PC_GS_LOWER, P.SPLIT_AI, P.STAGE_DIRK)])
def test_ragged_levels(name, pc, split, stage):
    # N = 104: levels 104, 52, 26 (single-stage) and 104, 52, 26, 13 (monolithic); no level is a multiple of a tile
    N, dt, nsteps = 104, 1e-3, 2
    kap = synth.grf_kappa(N, 5)
    u0, _ = synth.sine_modes_u0(N, 0)
    otab = {"radau3": OT.radau_iia(3), "alexander": OT.alexander()}[name]
    ptab = {"radau3": P.tableaux.radau_iia(3), "alexander": P.tableaux.alexander()}[name]
    _, stp = make(N, kap, ptab, dt, rtol=1e-12, precond=pc, splitting=split, stage_type=stage)
    u = dev(u0)
    stp.advance(u, nsteps)
    ref = step.run(N, kap, otab, dt, nsteps, u0)[-1]
    assert rel(host(u), ref) < 1e-10


def test_largest_stage_count():
    # s = 8 (the library's maximum): Radau IIA(8) with P_L and P_LD against the coupled direct solve
    N, dt = 32, 1e-2
    kap = synth.grf_kappa(N, 6)
    M, K = fem.assemble(N, kap)
    otab = OT.radau_iia(8)
    f = synth.random_stage_block(N, 8, 26).ravel()
    ref = step.CoupledLU(M, K, otab["A"], dt).solve(f)
    for pc in (P.PC_GS_LOWER, P.PC_RANA_LD):
        _, stp = make(N, kap, P.tableaux.radau_iia(8), dt, rtol=1e-12, precond=pc)
        x, st = stp.solve_stages(dev(f))
        assert rel(host(x), ref) < 1e-9
    with pytest.raises(P.IrkError):  # nine stages exceed the library's limit
        make(N, kap, P.tableaux.radau_iia(9), dt)


def test_empty_work():
    N, dt = 16, 1e-3
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), dt)
    u = dev(u0)
    rc, st = stp.advance(u, 0)
    assert rc == 0 and st["steps_done"] == 0 and np.array_equal(host(u), u0)
    x, st = stp.solve_stages(dev(np.zeros(3 * (N - 1) ** 2)))
    assert not np.any(host(x)) and st["fgmres_its_total"] == 0


def test_device_allocation_failure_reported_and_freed():
    # N = 16384 (the largest grid the library accepts), s = 3, restart 32: one stage vector is 3 (N+1) * pitch
    # doubles = 6.45 GB, so the Krylov basis V (33 vectors, 213 GB) fits in the 288 GB of HBM and the flexible
    # basis Z (32 vectors, 206 GB) after it cannot: creation must stop at Z with IRK_ENOMEM and free V again
    import torch

    N = 16384
    kap = torch.ones(N * N, dtype=torch.float64, device="cuda")
    prob = P.Problem(N, kap)
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    assert total < 420e9  # V and Z together exceed the device
    with pytest.raises(P.IrkError) as e:
        P.Stepper(prob, P.tableaux.radau_iia(3), 1e-3, restart=32)
    assert e.value.code == P.IRK_ENOMEM and "hipMalloc" in str(e.value)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (256 << 20)
    prob.close()
    del kap
    # the library is usable afterwards
    n = 16
    _, stp = make(n, np.ones(n * n), P.tableaux.radau_iia(3), 1e-3, rtol=1e-12)
    u0, amps = synth.sine_modes_u0(n, 0)
    u = dev(u0)
    stp.advance(u, 1)
    assert rel(host(u), step.closed_form_modes(n, OT.radau_iia(3), 1e-3, 1, amps)[1]) < 1e-10
