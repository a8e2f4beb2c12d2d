"""The exact stage-coupled Runge-Kutta step (FP64, CPU).

Test infrastructure only (see the package docstring).

For the linear problem M u' = -K u + F, one step of an s-stage Runge-Kutta
method (Section 2, eq:stageeq and the update y^{n+1} = y^n + dt sum b_i k_i, with
the mass matrix kept on the left) finds the stage derivatives k = (k_1..k_s),
stage-major, from the stage-coupled system of Section 3 (eq:block_struct_AI)

    (I_s (x) M + dt * A (x) K) k = f,      f_i = -K u^n + F_i,

and sets u^{n+1} = u^n + dt * sum_i b_i k_i. (eq:rkheat writes the heat equation
with "+", which fixes the sign typo of eq:heat; the update formula after
eq:rkheat drops the factor dt, which the general update of Section 2 carries.)

The system has exactly one solution whenever every eigenvalue of A has positive
real part, so the oracle computes it directly and does not imitate any
preconditioner. Four independent tiers:
  1. dense brute force (tiny grids),
  2. the full coupled sparse LU (SuperLU) -- the reference for N <= 512,
  3. an eigen-decoupled direct solve (A = V Lambda V^{-1} turns the system into s
     independent sparse systems M + dt*lambda_i*K) -- used where tier 2 does not
     fit in memory (1024^2),
  4. the closed form for constant kappa: discrete sine modes are generalized
     eigenvectors of (K, M), so u^n = sum_m alpha_m R(-dt lambda_m)^n v_m.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .tableaux import stability_function


def coupled_matrix(M, K, A, dt):
    """Stage-major coupled operator I_s (x) M + dt * A (x) K (eq:block_struct_AI)."""
    s = np.asarray(A).shape[0]
    return (sp.kron(sp.identity(s), M) + dt * sp.kron(sp.csr_matrix(np.asarray(A)), K)).tocsc()


def coupled_matrix_ia(M, K, A, dt):
    """Butcher's IA form A^{-1} (x) M + dt I_s (x) K (eq:block_struct_IA) acting on the stage combinations
    w = (A (x) I) k (eq:butcherw, eq:stageeqw); the right-hand side is the same f as in the AI form."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    return (sp.kron(sp.csr_matrix(np.linalg.inv(A)), M) + dt * sp.kron(sp.identity(s), K)).tocsc()


def stages_from_w(A, w):
    """k = (A^{-1} (x) I) w: undo eq:butcherw (one small solve with A for all nodes at once)."""
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    return np.linalg.solve(A, np.asarray(w).reshape(s, -1)).ravel()


def dirk_solve(M, K, A, dt, rhs, trans=False, lu=None):
    """Stage-by-stage solve of the coupled system for a lower-triangular A (Section 2.3, DIRK).

    (I (x) M + dt A (x) K) k = rhs is block lower triangular, so stage i needs one single-stage
    solve with M + dt a_ii K after moving the already known stages to the right:
        (M + dt a_ii K) k_i = rhs_i - dt K sum_{j<i} a_ij k_j.
    The transposed system (A^T upper triangular) runs backwards: j > i with a_ji.
    lu: optional dict that keeps one sparse LU factorisation per diagonal entry a_ii across calls
    (M and K are symmetric, so the transposed system uses the same blocks); without it every stage
    solve factorises its block afresh.
    """
    A = np.asarray(A, dtype=np.float64)
    s = A.shape[0]
    if np.any(np.triu(A, 1) != 0.0):
        raise ValueError("DIRK needs a lower-triangular A")
    R = np.asarray(rhs).reshape(s, -1)
    k = np.zeros_like(R)
    order = range(s - 1, -1, -1) if trans else range(s)
    for i in order:
        known = range(i + 1, s) if trans else range(i)
        t = R[i].copy()
        for j in known:
            aij = A[j, i] if trans else A[i, j]
            t -= dt * (K @ (aij * k[j]))
        if lu is None:
            k[i] = spla.spsolve((M + dt * A[i, i] * K).tocsc(), t)
        else:
            if A[i, i] not in lu:
                lu[A[i, i]] = spla.splu((M + dt * A[i, i] * K).tocsc())
            k[i] = lu[A[i, i]].solve(t)
    return k.ravel()


def stage_rhs(K, u, s, F=None):
    """Right-hand side f_i = -K u^n + F_i, identical for every stage when F is constant in time."""
    f = -(K @ u)
    if F is not None:
        f = f + F
    return np.tile(f, s)


def update(u, k, b, dt):
    """u^{n+1} = u^n + dt * sum_i b_i k_i (k stage-major, shape (s*n,))."""
    s = len(b)
    kk = np.asarray(k).reshape(s, -1)
    return u + dt * (np.asarray(b) @ kk)


class CoupledLU:
    """Tier 2: one SuperLU factorization of the full coupled operator.

    kappa, dt and A are fixed for a run, so one factorization serves every step.
    The factorization is applied to the node-major permutation of the
    stage-major operator (a symmetric permutation of rows and columns that keeps
    the fill low); solve() maps back. ``trans=True`` solves with the transpose,
    I (x) M + dt A^T (x) K.
    """

    def __init__(self, M, K, A, dt):
        s = np.asarray(A).shape[0]
        n = M.shape[0]
        self.s, self.n = s, n
        # node-major position of stage-major entry (i, p): p*s + i
        perm = (np.arange(s)[:, None] + s * np.arange(n)[None, :]).ravel()
        self.perm = perm
        Acal = coupled_matrix(M, K, A, dt)
        P = sp.csr_matrix((np.ones(s * n), (perm, np.arange(s * n))), shape=(s * n, s * n))
        self.lu = spla.splu((P @ Acal @ P.T).tocsc(), permc_spec="MMD_AT_PLUS_A")

    def solve(self, rhs, trans: bool = False):
        rp = np.empty_like(rhs)
        rp[self.perm] = rhs
        xp = self.lu.solve(rp, trans="T" if trans else "N")
        return xp[self.perm]


class DecoupledLU:
    """Tier 3: the eigen-decoupled direct solve.

    With A = V diag(lam) V^{-1}, (I (x) M + dt A (x) K) = (V (x) I)(I (x) M + dt diag(lam) (x) K)(V^{-1} (x) I),
    so each step is s independent sparse solves with M + dt*lam_i*K (complex for
    conjugate pairs of lam). An exact direct method, not the GPU algorithm.
    """

    def __init__(self, M, K, A, dt):
        A = np.asarray(A, dtype=np.float64)
        lam, V = np.linalg.eig(A)
        self.s = A.shape[0]
        self.n = M.shape[0]
        self.V = V
        self.Vinv = np.linalg.inv(V)
        self.lam = lam
        self.factors = []
        done = {}
        Mc = M.tocsc()
        Kc = K.tocsc()
        for i, l in enumerate(lam):
            key = None
            # a conjugate partner already factored? reuse its factor by conjugation
            for j, fj in done.items():
                if abs(lam[j] - np.conj(l)) < 1e-12 * max(1.0, abs(l)) and abs(l.imag) > 0:
                    key = j
            if key is not None:
                self.factors.append(("conj", key))
                continue
            if abs(l.imag) > 0:
                B = (Mc.astype(np.complex128) + dt * l * Kc.astype(np.complex128)).tocsc()
            else:
                B = (Mc + dt * l.real * Kc).tocsc()
            done[i] = spla.splu(B, permc_spec="MMD_AT_PLUS_A")
            self.factors.append(("own", i))
        self.lus = done

    def _block_solve(self, i, r):
        kind, j = self.factors[i]
        lu = self.lus[j]
        if kind == "own":
            if np.iscomplexobj(self.lam) and abs(self.lam[i].imag) > 0:
                return lu.solve(r.astype(np.complex128))
            if np.iscomplexobj(r):
                return lu.solve(r.real.copy()) + 1j * lu.solve(r.imag.copy())
            return lu.solve(r)
        # conj(M + dt*conj(l)*K)^{-1} conj(r) = ((M + dt*l*K)^{-1} r) conjugated
        return np.conj(lu.solve(np.conj(r).astype(np.complex128)))

    def solve(self, rhs, trans: bool = False):
        s, n = self.s, self.n
        R = np.asarray(rhs, dtype=np.float64).reshape(s, n)
        if trans:
            # (V (x) I)^{-T} ... : transpose swaps V and V^{-1}; the diagonal blocks are symmetric
            W = self.V.T @ R
            Y = np.stack([self._block_solve(i, W[i]) for i in range(s)])
            X = self.Vinv.T @ Y
        else:
            W = self.Vinv @ R
            Y = np.stack([self._block_solve(i, W[i]) for i in range(s)])
            X = self.V @ Y
        return np.real(X).ravel()


def dense_solve(M, K, A, dt, rhs):
    """Tier 1: dense brute-force solve of the coupled system."""
    Acal = coupled_matrix(M, K, A, dt).toarray()
    return np.linalg.solve(Acal, rhs)


def run(N, kappa, tab, dt, nsteps, u0, F=None, tier="coupled", return_stages=False, splitting="AI"):
    """Integrate nsteps steps; returns the list [u^0, u^1, ..., u^nsteps] (and the stage unknowns).

    tier: "coupled" (tier 2), "decoupled" (tier 3, AI only), "dense" (tier 1) or "dirk" (stage-by-stage
    single-stage solves for a lower-triangular A, AI only).
    splitting: "AI" solves eq:block_struct_AI for k; "IA" solves eq:block_struct_IA for w and
    recovers k = (A^{-1} (x) I) w for the update (the stage unknowns returned are then w).
    """
    M, K = fem.assemble(N, kappa)
    A = np.asarray(tab["A"])
    b = np.asarray(tab["b"])
    s = b.size
    if splitting not in ("AI", "IA"):
        raise ValueError(splitting)
    if splitting == "IA":
        if tier == "coupled":
            solver = spla.splu(coupled_matrix_ia(M, K, A, dt)).solve
        elif tier == "dense":
            Ad = coupled_matrix_ia(M, K, A, dt).toarray()
            solver = lambda r: np.linalg.solve(Ad, r)  # noqa: E731
        else:
            raise ValueError(tier)
    elif tier == "coupled":
        solver = CoupledLU(M, K, A, dt).solve
    elif tier == "decoupled":
        solver = DecoupledLU(M, K, A, dt).solve
    elif tier == "dense":
        Ad = coupled_matrix(M, K, A, dt).toarray()
        solver = lambda r, trans=False: np.linalg.solve(Ad.T if trans else Ad, r)  # noqa: E731
    elif tier == "dirk":
        factors = {}
        solver = lambda r: dirk_solve(M, K, A, dt, r, lu=factors)  # noqa: E731
    else:
        raise ValueError(tier)
    us = [np.asarray(u0, dtype=np.float64).copy()]
    ks = []
    u = us[0]
    for _ in range(nsteps):
        x = solver(stage_rhs(K, u, s, F))
        ks.append(x)
        k = stages_from_w(A, x) if splitting == "IA" else x
        u = update(u, k, b, dt)
        us.append(u)
    if return_stages:
        return us, ks
    return us


def discrete_eigenvalue(N, j, k):
    """Generalized eigenvalue of (K, M), kappa = 1, for the discrete mode sin(j pi x) sin(k pi y).

    The Q1 matrices are tensor products of the 1-D P1 matrices
    (1/h) tridiag(-1, 2, -1) and (h/6) tridiag(1, 4, 1), whose common
    eigenvectors are the sampled sines; the ratio of their symbols gives
    (6/h^2)(1 - cos t)/(2 + cos t) per direction.
    """
    h = 1.0 / N

    def one(m):
        t = m * np.pi * h
        return 6.0 / (h * h) * (1.0 - np.cos(t)) / (2.0 + np.cos(t))

    return one(j) + one(k)


def closed_form_modes(N, tab, dt, nsteps, amps):
    """Tier 4: u^n for u^0 = sum alpha_jk sin(j pi x) sin(k pi y), kappa = 1.

    Each mode is a generalized eigenvector of (K, M) with eigenvalue lam_jk, so the
    Runge-Kutta step multiplies its coefficient by R(-dt lam_jk).
    Returns the list [u^0, ..., u^nsteps].
    """
    from synth import sine_mode_vector

    amps = np.asarray(amps)
    out = []
    modes = []
    for j in range(1, amps.shape[0] + 1):
        for k in range(1, amps.shape[1] + 1):
            lam = discrete_eigenvalue(N, j, k)
            R = stability_function(tab, -dt * lam)[0].real
            modes.append((amps[j - 1, k - 1], R, sine_mode_vector(N, j, k)))
    for n in range(nsteps + 1):
        u = np.zeros((N - 1) * (N - 1))
        for a, R, v in modes:
            u += a * R**n * v
        out.append(u)
    return out


def closed_form_any(N, tab, dt, nsteps, u0):
    """Tier 4 for arbitrary u^0 with kappa = 1: expand u^0 in discrete sine modes (DST-I).

    Returns u^nsteps.
    """
    m = N - 1
    U = np.asarray(u0, dtype=np.float64).reshape(m, m)  # [j-1 (y), i-1 (x)]
    coef = scipy.fft.dstn(U, type=1) / (N * N)  # coefficient of sin(k pi y) sin(j pi x)
    jj = np.arange(1, N)
    h = 1.0 / N
    one = 6.0 / (h * h) * (1.0 - np.cos(jj * np.pi * h)) / (2.0 + np.cos(jj * np.pi * h))
    lam = one[:, None] + one[None, :]
    R = stability_function(tab, (-dt * lam).ravel()).real.reshape(lam.shape)
    coef_n = coef * R**nsteps
    return (scipy.fft.idstn(coef_n * (N * N), type=1)).ravel()
