"""Plain CSR statement of the stage preconditioners and the multigrid V-cycle (FP64, CPU).

Test infrastructure only (see the package docstring).

Section 3.1 (Block preconditioners) replaces the Butcher matrix A by a lower
triangular Atil: with the additive split A = L + D + U, Atil = D (block Jacobi,
eq:pcbjac) or L + D (block Gauss-Seidel, eq:pcbgs); with the multiplicative
factorisation A = L_1 D U_1 (unit triangular L_1, U_1), Atil = L_1 D (Rana-LD,
eq:pcranald). The paper states them for the form eq:block_struct_IA and notes that
the form eq:block_struct_AI "follows similarly"; the reading used here (the AI
form) is

    P = I (x) M + dt * Atil (x) K.

Applying P^{-1} to v is block forward substitution:
    t_i = v_i - dt * K * sum_{j<i} atil_ij z_j,    z_i = B_i^{-1} t_i,
with the diagonal blocks B_i = M + dt * atil_ii * K (the backward-Euler-like blocks
of Section 3.1, there written a_jj^{-1} M + dt K for the IA form). The paper
approximates B_i^{-1} by multigrid; this module states the geometric multigrid
V-cycle used for that:

  * levels N, N/2, ... halving while the element count is even and larger than
    `coarse_n`; the coarse problem is rediscretised with the per-element
    diffusivity averaged over the 4 children;
  * prolongation P = bilinear interpolation, restriction = P^T;
  * smoother: Chebyshev iteration of a given degree preconditioned by point
    Jacobi (for Q1 the vertex-patch additive Schwarz smoother of Section 3.2
    reduces to point Jacobi), on the interval [lo*mu, hi*mu] with mu the
    largest eigenvalue of D^{-1}B estimated by power iteration (the paper's
    relaxation uses [0.25 mu, 1.1 mu] with mu estimated, Section 4.3);
  * coarsest level: a direct solve (the paper uses a direct method on the
    coarsest grid, Section 4.3).

Power iteration start vectors come from the SplitMix64 generator (Steele, Lea &
Flood, OOPSLA 2014), written here from its published definition; the GPU library
carries its own implementation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem

MASK64 = (1 << 64) - 1


def splitmix64(z: int) -> int:
    """One output of SplitMix64 for the counter value z (Steele, Lea & Flood 2014)."""
    z = (z + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def start_vector(n: int, level: int) -> np.ndarray:
    """Power-iteration start vector: entry p is 2*U - 1, U = top 53 bits of splitmix64(p + level*2^32) / 2^53.

    Vectorised with wrapping uint64 arithmetic; :func:`splitmix64` is the scalar statement.
    """
    z = np.arange(n, dtype=np.uint64) + np.uint64(level << 32)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)) - 1.0


def level_sizes(N: int, coarse_n: int = 32):
    """Element counts per side of the multigrid levels, finest first."""
    sizes = [N]
    while sizes[-1] % 2 == 0 and sizes[-1] > coarse_n:
        sizes.append(sizes[-1] // 2)
    return sizes


def coarsen_kappa(N: int, kappa: np.ndarray) -> np.ndarray:
    """Per-element diffusivity of the next level: the mean of the 4 children."""
    k = np.asarray(kappa).reshape(N, N)
    kc = 0.25 * (k[0::2, 0::2] + k[0::2, 1::2] + k[1::2, 0::2] + k[1::2, 1::2])
    return kc.ravel()


def prolongation(Nc: int) -> sp.csr_matrix:
    """Bilinear interpolation from the interior nodes of an Nc grid to those of the 2*Nc grid.

    Fine node (i, j) receives w(i - 2I) w(j - 2J) of coarse node (I, J), with
    w(0) = 1, w(+-1) = 1/2. Coarse boundary nodes carry zero.
    """
    Nf = 2 * Nc
    fidx = fem.interior_index(Nf)
    cidx = fem.interior_index(Nc)
    rows, cols, vals = [], [], []
    w = {0: 1.0, 1: 0.5, -1: 0.5}
    for J in range(1, Nc):
        for I in range(1, Nc):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    i, j = 2 * I + di, 2 * J + dj
                    rows.append(fidx[j, i])
                    cols.append(cidx[J, I])
                    vals.append(w[di] * w[dj])
    nf = (Nf - 1) ** 2
    nc = (Nc - 1) ** 2
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def chebyshev_smooth(B, Dinv, t, x0, lo, hi, degree):
    """Jacobi-preconditioned Chebyshev iteration on [lo, hi] (Saad, Iterative Methods, Alg. 12.1).

    theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta.
      r_0 = t - B x_0, rho_0 = 1/sigma, d_0 = D^{-1} r_0 / theta
      x_{k+1} = x_k + d_k
      r_{k+1} = t - B x_{k+1}, rho_{k+1} = 1/(2 sigma - rho_k)
      d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^{-1} r_{k+1}
    Returns x_degree (degree operator applications in total).
    """
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    x = np.array(x0, dtype=np.float64, copy=True)
    r = t - B @ x
    rho = 1.0 / sigma
    d = Dinv * r / theta
    for k in range(degree):
        x = x + d
        if k + 1 == degree:
            break
        r = t - B @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv * r)
        rho = rho_new
    return x


def power_mu(B, Dinv, level: int, iters: int) -> float:
    """Estimate of the largest eigenvalue of D^{-1} B by `iters` power iterations.

    x <- D^{-1} B x / |D^{-1} B x|_2 from the SplitMix64 start vector, then the
    Rayleigh quotient x^T B x / x^T D x of the symmetric pencil (B, D).
    """
    x = start_vector(B.shape[0], level)
    for _ in range(iters):
        y = Dinv * (B @ x)
        x = y / np.linalg.norm(y)
    return float((x @ (B @ x)) / (x @ (x / Dinv)))


class Hierarchy:
    """Multigrid hierarchy for the blocks B(a) = M + dt*a*K on all levels.

    Options mirror the GPU library's: coarse_n, cheb_degree, cheb_lo, cheb_hi,
    power_its.
    """

    def __init__(self, N, kappa, dt, coarse_n=32, cheb_degree=2, cheb_lo=0.25, cheb_hi=1.1, power_its=15):
        self.N = N
        self.dt = dt
        self.sizes = level_sizes(N, coarse_n)
        self.deg = cheb_degree
        self.lo = cheb_lo
        self.hi = cheb_hi
        self.power_its = power_its
        self.M, self.K, self.P = [], [], []
        kap = np.asarray(kappa, dtype=np.float64) if kappa is not None else np.ones(N * N)
        for l, Nl in enumerate(self.sizes):
            M, K = fem.assemble(Nl, kap)
            self.M.append(M)
            self.K.append(K)
            if l + 1 < len(self.sizes):
                self.P.append(prolongation(self.sizes[l + 1]))
                kap = coarsen_kappa(Nl, kap)
        self._blocks = {}

    def block(self, a: float, c: float = 1.0):
        """Per-level operators for one diagonal block B = c*M + dt*a*K: (B, Dinv, mu) lists and the coarse
        Cholesky factor. c = 1 is the AI-form block; c = 1/atil_ii, a = 1 the IA-form block."""
        key = (float(a), float(c))
        if key not in self._blocks:
            Bs, Dinvs, mus = [], [], []
            for l in range(len(self.sizes)):
                B = (c * self.M[l] + self.dt * a * self.K[l]).tocsr()
                Dinv = 1.0 / B.diagonal()
                Bs.append(B)
                Dinvs.append(Dinv)
                mus.append(power_mu(B, Dinv, l, self.power_its) if l + 1 < len(self.sizes) else None)
            chol = sla.cho_factor(Bs[-1].toarray(), lower=True)
            self._blocks[key] = (Bs, Dinvs, mus, chol)
        return self._blocks[key]

    def vcycle(self, a: float, t: np.ndarray, level: int = 0, c: float = 1.0) -> np.ndarray:
        """One V-cycle for (c*M + dt*a*K) x = t with zero initial guess on `level`."""
        Bs, Dinvs, mus, chol = self.block(a, c)
        if level == len(self.sizes) - 1:
            return sla.cho_solve(chol, t)
        B, Dinv, mu = Bs[level], Dinvs[level], mus[level]
        lo, hi = self.lo * mu, self.hi * mu
        x = chebyshev_smooth(B, Dinv, t, np.zeros_like(t), lo, hi, self.deg)
        r = t - B @ x
        P = self.P[level]
        e = self.vcycle(a, P.T @ r, level + 1, c)
        x = x + P @ e
        x = chebyshev_smooth(B, Dinv, t, x, lo, hi, self.deg)
        return x


def ldu(A):
    """A = L1 diag(D) U1 with unit lower L1 and unit upper U1 (Gaussian elimination without pivoting)."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    L1, U1, D = np.eye(s), np.eye(s), np.zeros(s)
    W = A.copy()
    for k in range(s):
        D[k] = W[k, k]
        if D[k] == 0.0:
            raise ValueError("zero pivot: A has no LDU factorisation without pivoting")
        for i in range(k + 1, s):
            L1[i, k] = W[i, k] / D[k]
            U1[k, i] = W[k, i] / D[k]
        for i in range(k + 1, s):
            for j in range(k + 1, s):
                W[i, j] -= L1[i, k] * D[k] * U1[k, j]
    return L1, D, U1


def preconditioner_matrix(kind, A):
    """Atil of the stage preconditioner (Section 3.1): D (P_D), L + D (P_L), U + D (P_U), or L1 D (P_LD).

    The same Atil serves both splittings: I (x) M + dt Atil (x) K for the AI form and
    Atil^{-1} (x) M + dt I (x) K for the IA form."""
    A = np.asarray(A, dtype=np.float64)
    if kind == "jacobi":
        return np.diag(np.diag(A))
    if kind == "gs_lower":
        return np.tril(A)
    if kind == "gs_upper":
        return np.triu(A)
    if kind == "rana_ld":
        L1, D, _ = ldu(A)
        return L1 @ np.diag(D)
    raise ValueError(kind)


def _upper(kind, trans):
    # gs_upper's Atil is upper triangular, the others lower (or diagonal); transposing swaps the two
    return (kind == "gs_upper") != bool(trans)


def apply_block_preconditioner(kind, A, dt, K, v, block_solve, trans=False):
    """Apply P^{-1} for the AI-form stage preconditioner P = I (x) M + dt Atil (x) K, or with
    trans=True its transpose P^T = I (x) M + dt Atil^T (x) K (M, K symmetric), the preconditioner of
    the transposed system I (x) M + dt A^T (x) K.

    kind: "jacobi" (P_D), "gs_lower" (P_L), "gs_upper" (P_U) or "rana_ld" (P_LD); v is
    stage-major (s*n,). Atil is triangular, so P is block triangular and is inverted by
    block substitution: forward (i = 0, 1, ...) for a lower Atil, backward for an upper one,
        z_i = B_i^{-1} (v_i - dt K sum_{j already solved} atil_ij z_j).
    block_solve(i, t) must return (an approximation of) B_i^{-1} t with
    B_i = M + dt*atil_ii*K (the diagonal is the same for Atil^T).
    """
    Atil = preconditioner_matrix(kind, A)
    if trans:
        Atil = Atil.T
    s = Atil.shape[0]
    order = range(s - 1, -1, -1) if _upper(kind, trans) else range(s)
    V = np.asarray(v).reshape(s, -1)
    Z = np.zeros_like(V)
    done = []
    for i in order:
        t = V[i].copy()
        if done and kind != "jacobi":
            w = np.zeros_like(t)
            for j in done:
                w += Atil[i, j] * Z[j]
            t = t - dt * (K @ w)
        Z[i] = block_solve(i, t)
        done.append(i)
    return Z.ravel()


def _diagonal(A):
    A = np.asarray(A, dtype=np.float64)
    return np.diag(A) if A.ndim == 2 else A


def exact_block_solver(M, K, A, dt):
    """block_solve inverting every diagonal block M + dt*d_i*K exactly (sparse LU); A is Atil or its diagonal."""
    d = _diagonal(A)
    lus = [spla.splu((M + dt * d[i] * K).tocsc()) for i in range(d.size)]
    return lambda i, t: lus[i].solve(t)


def vcycle_block_solver(hier: Hierarchy, A):
    """block_solve applying one V-cycle of `hier` to every diagonal block; A is Atil or its diagonal."""
    d = _diagonal(A)
    return lambda i, t: hier.vcycle(d[i], t)


# ---------------------------------------------------------------- IA form (eq:block_struct_IA)


def apply_ia_block_preconditioner(kind, A, dt, M, K, v, block_solve, trans=False):
    """Apply P^{-1} for the IA-form stage preconditioner P = Atil^{-1} (x) M + dt I (x) K
    (eq:pcbjac, eq:pcbgs, eq:pcranald as printed, for eq:block_struct_IA), or with trans=True its
    transpose Atil^{-T} (x) M + dt I (x) K.

    Atil is triangular, so C = Atil^{-1} is triangular too and P is block triangular with diagonal
    blocks c_ii M + dt K (c_ii = 1/atil_ii); the stages are coupled through M:
        z_i = B_i^{-1} (v_i - M sum_{j already solved} c_ij z_j).
    block_solve(i, t) must return (an approximation of) (c_ii M + dt K)^{-1} t.
    """
    Atil = preconditioner_matrix(kind, A)
    if trans:
        Atil = Atil.T
    C = np.linalg.inv(Atil)
    s = Atil.shape[0]
    order = range(s - 1, -1, -1) if _upper(kind, trans) else range(s)
    V = np.asarray(v).reshape(s, -1)
    Z = np.zeros_like(V)
    done = []
    for i in order:
        t = V[i].copy()
        if done and kind != "jacobi":
            w = np.zeros_like(t)
            for j in done:
                w += C[i, j] * Z[j]
            t = t - M @ w
        Z[i] = block_solve(i, t)
        done.append(i)
    return Z.ravel()


def exact_ia_block_solver(M, K, Atil, dt):
    """block_solve inverting every IA diagonal block (1/atil_ii) M + dt K exactly (sparse LU)."""
    d = _diagonal(Atil)
    lus = [spla.splu(((1.0 / d[i]) * M + dt * K).tocsc()) for i in range(d.size)]
    return lambda i, t: lus[i].solve(t)


def vcycle_ia_block_solver(hier: Hierarchy, Atil):
    """block_solve applying one V-cycle of `hier` to every IA diagonal block (1/atil_ii) M + dt K."""
    d = _diagonal(Atil)
    return lambda i, t: hier.vcycle(1.0, t, c=1.0 / d[i])
