"""Monolithic multigrid for the stage-coupled system (Section 3.2), plain CSR statement (FP64, CPU).

Test infrastructure only (see the package docstring).

Instead of decoupling the stages, the multigrid cycle acts on the whole coupled
operator. For the AI form (eq:block_struct_AI) and the IA form (eq:block_struct_IA)
alike, a level operator is written

    Acal_l = Cm (x) M_l + dt * Ck (x) K_l,     (Cm, Ck) = (I, A) for AI, (A^{-1}, I) for IA,

and the transposed system uses (Cm^T, Ck^T). The relaxation is the additive Schwarz
method of eq:Cinv on the stage-coupled decomposition eq:bigdecomp: every patch
V_v x ... x V_v holds the s stage values of one vertex v (for Q1 on H^1 a vertex
patch is a single node, so the scalar method is point Jacobi), so

    C^{-1} r = sum_v p_v A_v^{-1} r_v,   A_v = p_v^T Acal p_v = Cm M_vv + dt Ck K_vv (s x s).

As in the single-stage cycle (oracle.mg), the relaxation is accelerated by a
Chebyshev iteration on [lo*mu, hi*mu] (the Section 4.3 setting), mu estimated by
power iteration on C^{-1} Acal from the SplitMix64 start vector of length s*n
(stage-major) followed by the quotient x^T Acal x / x^T C x, which for s = 1 is
the single-stage estimate. Transfers are I (x) P and I (x) P^T, coarse operators
are rediscretised, and the coarsest level is solved directly.

Levels: halve while the element count is even and either larger than `coarse_n`
or the coupled coarsest system would exceed `max_coarse` unknowns.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem
from .mg import coarsen_kappa, prolongation, start_vector


def mixing(A, splitting="AI", trans=False):
    """(Cm, Ck) of the level operator Cm (x) M + dt Ck (x) K for the AI or IA form (or its transpose)."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    if splitting == "AI":
        Cm, Ck = np.eye(s), A.copy()
    elif splitting == "IA":
        Cm, Ck = np.linalg.inv(A), np.eye(s)
    else:
        raise ValueError(splitting)
    if trans:
        Cm, Ck = Cm.T.copy(), Ck.T.copy()
    return Cm, Ck


def level_sizes(N: int, s: int, coarse_n: int = 32, max_coarse: int = 1024):
    sizes = [N]
    while sizes[-1] % 2 == 0 and (sizes[-1] > coarse_n or s * (sizes[-1] - 1) ** 2 > max_coarse):
        sizes.append(sizes[-1] // 2)
    return sizes


def coupled_level_matrix(M, K, Cm, Ck, dt):
    return (sp.kron(sp.csr_matrix(Cm), M) + dt * sp.kron(sp.csr_matrix(Ck), K)).tocsr()


def patch_blocks(M, K, Cm, Ck, dt):
    """A_v = Cm M_vv + dt Ck K_vv for every interior vertex v: array (n, s, s)."""
    mv = M.diagonal()
    kv = K.diagonal()
    return mv[:, None, None] * Cm[None, :, :] + dt * kv[:, None, None] * Ck[None, :, :]


def additive_schwarz(blocks, r):
    """eq:Cinv on the vertex-times-stages patches: z_v = A_v^{-1} r_v (r, z stage-major)."""
    n, s, _ = blocks.shape
    R = np.asarray(r).reshape(s, n).T  # (n, s): the patch restriction r_v
    Z = np.linalg.solve(blocks, R[:, :, None])[:, :, 0]
    return Z.T.ravel()


def patch_energy(blocks, x):
    """x^T C x = sum_v x_v^T A_v x_v."""
    n, s, _ = blocks.shape
    X = np.asarray(x).reshape(s, n).T
    return float(np.einsum("vi,vij,vj->", X, blocks, X))


class MonolithicHierarchy:
    """Monolithic V-cycle for Cm (x) M + dt Ck (x) K on all levels (options mirror the single-stage cycle)."""

    def __init__(self, N, kappa, dt, Cm, Ck, coarse_n=32, cheb_degree=2, cheb_lo=0.25, cheb_hi=1.1, power_its=15,
                 max_coarse=1024):
        self.Cm = np.asarray(Cm, dtype=np.float64)
        self.Ck = np.asarray(Ck, dtype=np.float64)
        self.s = self.Cm.shape[0]
        self.dt = dt
        self.sizes = level_sizes(N, self.s, coarse_n, max_coarse)
        self.deg = cheb_degree
        self.lo, self.hi = cheb_lo, cheb_hi
        self.ops, self.blocks, self.P, self.mus = [], [], [], []
        kap = np.asarray(kappa, dtype=np.float64) if kappa is not None else np.ones(N * N)
        for l, Nl in enumerate(self.sizes):
            M, K = fem.assemble(Nl, kap)
            A = coupled_level_matrix(M, K, self.Cm, self.Ck, dt)
            self.ops.append(A)
            self.blocks.append(patch_blocks(M, K, self.Cm, self.Ck, dt))
            if l + 1 < len(self.sizes):
                self.P.append(sp.kron(sp.identity(self.s), prolongation(self.sizes[l + 1])).tocsr())
                kap = coarsen_kappa(Nl, kap)
                self.mus.append(self._power_mu(l, power_its))
        self.coarse_lu = sla.lu_factor(self.ops[-1].toarray())

    def _power_mu(self, l, iters):
        A, blk = self.ops[l], self.blocks[l]
        x = start_vector(A.shape[0], l)
        for _ in range(iters):
            y = additive_schwarz(blk, A @ x)
            x = y / np.linalg.norm(y)
        return float((x @ (A @ x)) / patch_energy(blk, x))

    def smooth(self, l, t, x0):
        """Chebyshev iteration (Saad, Alg. 12.1) preconditioned by the additive Schwarz relaxation."""
        A, blk, mu = self.ops[l], self.blocks[l], self.mus[l]
        lo, hi = self.lo * mu, self.hi * mu
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        sigma = theta / delta
        x = np.array(x0, dtype=np.float64, copy=True)
        r = t - A @ x
        rho = 1.0 / sigma
        d = additive_schwarz(blk, r) / theta
        for k in range(self.deg):
            x = x + d
            if k + 1 == self.deg:
                break
            r = t - A @ x
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * additive_schwarz(blk, r)
            rho = rho_new
        return x

    def vcycle(self, t, level=0):
        """One monolithic V-cycle for Acal x = t (stage-major) with zero initial guess."""
        if level == len(self.sizes) - 1:
            return sla.lu_solve(self.coarse_lu, t)
        x = self.smooth(level, t, np.zeros_like(t))
        r = t - self.ops[level] @ x
        P = self.P[level]
        x = x + P @ self.vcycle(P.T @ r, level + 1)
        return self.smooth(level, t, x)
