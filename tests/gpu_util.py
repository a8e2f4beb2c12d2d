"""Helpers shared by the GPU parity tests (device transfers, relative errors)."""
import numpy as np


def dev(x):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make(N, kappa, tab, dt, **opts):
    import paper_2403_08084_amd as P

    prob = P.Problem(N, dev(kappa))
    return prob, P.Stepper(prob, tab, dt, **opts)
