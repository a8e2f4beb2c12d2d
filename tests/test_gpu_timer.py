"""GPU: the measurement hook behind bench.py's roofline (irk_kernel_timer). It must time every dispatch of the
step's kernel families, charge each the algorithmic bytes stated for its kernel, and leave the results unchanged."""
import numpy as np
import pytest

import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host, make

pytestmark = pytest.mark.gpu


def _run(N, prec, timer):
    kap = synth.grf_kappa(N, 1)
    u0, _ = synth.sine_modes_u0(N, 0)
    _, stp = make(N, kap, P.tableaux.radau_iia(3), 1e-3, mg_precision=prec, rtol=1e-10)
    if timer:
        stp.kernel_timer(P.KFAM_ALL, True)
    u = dev(u0)
    _, st = stp.advance(u, 2)
    return stp, st, host(u)


@pytest.mark.parametrize("prec", [P.F32, P.F64])
def test_timer_accounts_every_family(prec):
    N, s = 128, 3
    n = (N - 1) ** 2
    stp, st, u_t = _run(N, prec, True)
    fam = {f: stp.kernel_timer_family(f) for f in range(len(P.KFAM_NAMES))}
    cycles = st["fgmres_its_total"] + st["arnoldi_discarded"]  # preconditioner applications (eager: no graphs)
    # every family that runs on this path was timed, and only those
    for f in (P.KFAM_GRAM_SCHMIDT, P.KFAM_OPERATOR, P.KFAM_MG_FINE, P.KFAM_MG_COARSE, P.KFAM_COARSE_SOLVE,
              P.KFAM_REDUCE_FINISH, P.KFAM_OTHER):
        launches, ms, by, bmin = fam[f]
        assert launches > 0 and ms > 0, P.KFAM_NAMES[f]
        assert bmin <= by + 1e-6
    # one finest DOWN and one finest UP per stage V-cycle, s V-cycles per preconditioner application
    assert fam[P.KFAM_MG_FINE][0] == 2 * s * cycles
    # the stage operator's bytes: the s input planes (vectors of the flexible basis: FP32 in the mixed form, FP64
    # otherwise), s FP64 output planes and the FP64 diffusivity; the true-residual check that ends every restart
    # cycle of every solve reads an FP64 input and the right-hand side's s planes besides
    launches, _, by, _ = fam[P.KFAM_OPERATOR]
    residuals = st["solves"] + st["restarts_total"]
    assert launches == cycles + residuals
    zb = 4 if prec != P.F64 else 8
    assert by == pytest.approx((cycles * (zb * s + 8 * s + 8) + residuals * (24 * s + 8)) * n, rel=1e-12)
    # the aggregate is the sum of the families
    tot = stp.kernel_timer_family(P.KFAM_ALL)
    assert tot[0] == sum(v[0] for v in fam.values())
    assert tot[2] == pytest.approx(sum(v[2] for v in fam.values()), rel=1e-12)
    # timing the dispatches changes nothing in the result
    _, _, u_plain = _run(N, prec, False)
    assert np.array_equal(u_t, u_plain)
