"""Q1 finite elements on a uniform N x N grid of the unit square (FP64, CPU).

Test infrastructure only (see the package docstring).

The semidiscrete heat / diffusion problem of Section 2 (the heat equation and its
Runge-Kutta stage form, eq:heat and eq:rkheat) is written M u' = -K u + f, with
M the consistent mass matrix and K the stiffness matrix of div(kappa grad u).
Homogeneous Dirichlet data are imposed as in Section 2.1 ("DAE-type" boundary
conditions): with g = 0 and an invertible Butcher matrix the stage values on the
boundary vanish, so boundary rows and columns are simply removed.

Node numbering: node (i, j) at (i/N, j/N); interior nodes 1 <= i, j <= N-1 are
numbered (j-1)*(N-1) + (i-1). Element (ex, ey) covers [ex/N,(ex+1)/N] x
[ey/N,(ey+1)/N] and carries kappa[ey*N + ex]. Local element node order:
(0,0), (1,0), (1,1), (0,1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Local node offsets (dx, dy) in the order (0,0), (1,0), (1,1), (0,1).
LOCAL_NODES = ((0, 0), (1, 0), (1, 1), (0, 1))


def _gauss_2pt():
    """Two-point Gauss-Legendre rule on [0, 1] (exact for cubics per direction)."""
    g = 0.5 / np.sqrt(3.0)
    return np.array([0.5 - g, 0.5 + g]), np.array([0.5, 0.5])


def _bilinear(xi, eta):
    """Bilinear basis values and reference gradients at (xi, eta) in [0,1]^2."""
    phi = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
    dxi = np.array([-(1 - eta), (1 - eta), eta, -eta])
    deta = np.array([-(1 - xi), -xi, xi, (1 - xi)])
    return phi, dxi, deta


def element_matrices(h: float):
    """Element stiffness (kappa = 1) and mass matrices of a square of side h.

    Integrals of grad(phi_a).grad(phi_b) and phi_a*phi_b over the element,
    evaluated with the 2x2 Gauss rule (exact for bilinear products). In 2-D the
    stiffness matrix does not depend on h; the mass matrix scales with h^2.
    """
    pts, wts = _gauss_2pt()
    Ke = np.zeros((4, 4))
    Me = np.zeros((4, 4))
    for xi, wx in zip(pts, wts):
        for eta, wy in zip(pts, wts):
            phi, dxi, deta = _bilinear(xi, eta)
            w = wx * wy * h * h  # Jacobian of the map to the physical square
            gx = dxi / h
            gy = deta / h
            Ke += w * (np.outer(gx, gx) + np.outer(gy, gy))
            Me += w * np.outer(phi, phi)
    return Ke, Me


def interior_index(N: int) -> np.ndarray:
    """(N+1) x (N+1) array (indexed [j, i]) of interior dof numbers, -1 on the boundary."""
    idx = -np.ones((N + 1, N + 1), dtype=np.int64)
    m = N - 1
    jj, ii = np.meshgrid(np.arange(1, N), np.arange(1, N), indexing="ij")
    idx[jj, ii] = (jj - 1) * m + (ii - 1)
    return idx


def assemble(N: int, kappa=None):
    """Assemble the interior-node mass matrix M and stiffness matrix K(kappa).

    Standard element-by-element assembly: every element adds kappa_e * Ke and Me
    into the rows/columns of its four nodes; entries touching a boundary node are
    discarded (homogeneous Dirichlet elimination). Returns (M, K) as CSR, n x n
    with n = (N-1)^2.
    """
    h = 1.0 / N
    if kappa is None:
        kappa = np.ones(N * N)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(N, N)  # [ey, ex]
    Ke, Me = element_matrices(h)
    idx = interior_index(N)
    ey, ex = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ey = ey.ravel()
    ex = ex.ravel()
    kap = kappa[ey, ex]
    glob = [idx[ey + dy, ex + dx] for (dx, dy) in LOCAL_NODES]
    rows, cols, kv, mv = [], [], [], []
    for a in range(4):
        for b in range(4):
            ra, cb = glob[a], glob[b]
            keep = (ra >= 0) & (cb >= 0)
            rows.append(ra[keep])
            cols.append(cb[keep])
            kv.append(kap[keep] * Ke[a, b])
            mv.append(np.full(int(keep.sum()), Me[a, b]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    n = (N - 1) * (N - 1)
    K = sp.csr_matrix((np.concatenate(kv), (rows, cols)), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv), (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    M.sum_duplicates()
    return M, K


def assemble_full(N: int, kappa=None):
    """Assemble M and K over all (N+1)^2 nodes (no boundary elimination).

    Used only to check invariants of the assembly (zero row sums of the Neumann
    stiffness matrix, total mass equal to the area).
    """
    h = 1.0 / N
    if kappa is None:
        kappa = np.ones(N * N)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(N, N)
    Ke, Me = element_matrices(h)
    ey, ex = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ey = ey.ravel()
    ex = ex.ravel()
    kap = kappa[ey, ex]
    glob = [(ey + dy) * (N + 1) + (ex + dx) for (dx, dy) in LOCAL_NODES]
    rows, cols, kv, mv = [], [], [], []
    for a in range(4):
        for b in range(4):
            rows.append(glob[a])
            cols.append(glob[b])
            kv.append(kap * Ke[a, b])
            mv.append(np.full(ex.size, Me[a, b]))
    n = (N + 1) * (N + 1)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    K = sp.csr_matrix((np.concatenate(kv), (rows, cols)), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv), (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    M.sum_duplicates()
    return M, K


def element_gather(N: int, vec: np.ndarray) -> np.ndarray:
    """Values of an interior nodal vector at the 4 local nodes of every element.

    Returns an (N*N, 4) array in element layout; boundary nodes contribute 0.
    """
    idx = interior_index(N)
    ext = np.concatenate([np.asarray(vec, dtype=np.float64), [0.0]])
    ey, ex = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ey = ey.ravel()
    ex = ex.ravel()
    out = np.empty((N * N, 4))
    for a, (dx, dy) in enumerate(LOCAL_NODES):
        g = idx[ey + dy, ex + dx]
        out[:, a] = ext[np.where(g >= 0, g, -1)]
    return out
