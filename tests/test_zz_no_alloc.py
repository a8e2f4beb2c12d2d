"""GPU: the allocation-free mass entry point (irk_apply_mass_noalloc) against irk_apply_mass, through the C ABI.

Both run the same kernels, so the results must agree bit for bit; two calls in a row, the second on a smaller
grid, check that the shared static staging array carries nothing from one call into the next."""
import ctypes

import numpy as np
import pytest

from oracle import fem
import paper_2403_08084_amd as P
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _call(name, prob, x, y):
    import torch

    fn = getattr(P.lib(), name)
    rc = fn(prob._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


def test_apply_mass_noalloc_matches_apply_mass():
    import torch

    for N, seed in ((1024, 5), (256, 6)):
        prob = P.Problem(N, dev(synth.grf_kappa(N, 1)))
        x = dev(synth.random_stage_block(N, 1, seed).ravel())
        y_ref = torch.full_like(x, np.nan)
        y = torch.full_like(x, np.nan)
        assert _call("irk_apply_mass", prob, x, y_ref) == P.IRK_OK
        assert _call("irk_apply_mass_noalloc", prob, x, y) == P.IRK_OK
        torch.cuda.synchronize()
        print(f"N={N}: noalloc vs apply_mass max |diff| {float((y - y_ref).abs().max()):.3e}", flush=True)
        assert torch.equal(y, y_ref)
        if N <= 256:
            M, _ = fem.assemble(N, None)
            ref = M @ host(x)
            assert np.linalg.norm(host(y) - ref) <= 1e-14 * np.linalg.norm(ref)


def test_apply_mass_noalloc_rejects_large_grid():
    import torch

    N = 1040
    prob = P.Problem(N, dev(np.ones(N * N)))
    x = torch.zeros((N - 1) ** 2, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    assert _call("irk_apply_mass_noalloc", prob, x, y) == P.IRK_EINVAL
    assert b"N <= 1024" in P.lib().irk_last_error()
