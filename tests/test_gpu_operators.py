"""GPU parity: Q1 mass/stiffness, stage right-hand side (a1) and stage operator (a2) vs the oracle CSR."""
import numpy as np
import pytest

from oracle import fem, step
from oracle import tableaux as OT
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [8, 33, 96, 130])
def test_mass_and_stiffness(N):
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    x = np.random.default_rng(N).standard_normal((N - 1) ** 2)
    prob = P.Problem(N, dev(kap))
    assert rel(host(prob.apply_mass(dev(x))), M @ x) < 1e-14
    assert rel(host(prob.apply_stiffness(dev(x))), K @ x) < 1e-14


@pytest.mark.parametrize("N,s", [(32, 2), (96, 3), (40, 4)])
def test_stage_rhs(N, s):
    kap = synth.grf_kappa(N, 2)
    _, K = fem.assemble(N, kap)
    tab = P.tableaux.radau_iia(s) if s < 4 else P.tableaux.gauss_legendre(4)
    _, stp = make(N, kap, tab, 1e-3)
    rng = np.random.default_rng(3)
    u, F = rng.standard_normal((2, (N - 1) ** 2))
    assert rel(host(stp.stage_rhs(dev(u))), step.stage_rhs(K, u, s)) < 1e-14
    assert rel(host(stp.stage_rhs(dev(u), dev(F))), step.stage_rhs(K, u, s, F)) < 1e-14


@pytest.mark.parametrize("N,name,dt", [(32, "radau3", 1e-3), (96, "gl4", 5e-4), (40, "radau2", 1.0 / 32),
                                       (256, "radau3", 1e-3), (64, "lobatto", 0.1)])
@pytest.mark.parametrize("transpose", [False, True])
def test_stage_operator(N, name, dt, transpose):
    tabs = {"radau3": (P.tableaux.radau_iia(3), OT.radau_iia(3)), "gl4": (P.tableaux.gauss_legendre(4), OT.gauss_legendre(4)),
            "radau2": (P.tableaux.radau_iia(2), OT.radau_iia(2)), "lobatto": (P.tableaux.lobatto_iiic2(), OT.lobatto_iiic2())}
    ptab, otab = tabs[name]
    kap = synth.grf_kappa(N, 1)
    M, K = fem.assemble(N, kap)
    A = otab["A"].T if transpose else otab["A"]
    Acal = step.coupled_matrix(M, K, A, dt)
    _, stp = make(N, kap, ptab, dt)
    x = synth.random_stage_block(N, stp.s, 5).ravel()
    y = host(stp.apply_stage_operator(dev(x), transpose=transpose))
    assert rel(y, Acal @ x) < 1e-14


@pytest.mark.parametrize("n,xoff,yoff", [(0, 0, 0), (1, 0, 0), (7, 0, 0), (1_000_001, 0, 0), (1_000_000, 1, 0),
                                         (33, 0, 1), (64, 1, 1)])
def test_device_copy(n, xoff, yoff):
    # the measurement reference copy: exact for even and odd lengths, aligned (16-byte path) and offset by one
    # value (scalar path); nothing outside y is written; overlapping vectors are refused
    import torch

    src = torch.as_tensor(np.random.default_rng(n).standard_normal(n + 2)).cuda()
    dst = torch.full((n + 2,), -7.0, dtype=torch.float64, device="cuda")
    x, y = src[xoff:xoff + n], dst[yoff:yoff + n]
    P.device_copy(x, y)
    d = host(dst)
    assert np.array_equal(d[yoff:yoff + n], host(src)[xoff:xoff + n])
    assert np.all(d[:yoff] == -7.0) and np.all(d[yoff + n:] == -7.0)
    if n >= 2:
        with pytest.raises(P.IrkError) as e:
            P.device_copy(src[0:n - 1], src[1:n])
        assert e.value.code == P.IRK_EINVAL
