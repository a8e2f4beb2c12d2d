"""Pins for oracle.fem: element matrices, spectrum, invariants, stencils."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem
import synth


def test_element_matrices_closed_form():
    Ke, Me = fem.element_matrices(0.25)
    Kc = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    Mc = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) * 0.25**2 / 36.0
    assert np.abs(Ke - Kc).max() < 1e-15
    assert np.abs(Me - Mc).max() < 1e-17


def _one(N, m):
    h = 1.0 / N
    t = m * np.pi * h
    return 6.0 / h**2 * (1 - np.cos(t)) / (2 + np.cos(t))


def test_generalized_spectrum_closed_form():
    N = 8
    M, K = fem.assemble(N)
    ev = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    cf = np.sort([_one(N, j) + _one(N, k) for j in range(1, N) for k in range(1, N)])
    assert np.abs(ev - cf).max() < 1e-12 * cf.max()


@pytest.mark.parametrize("j,k", [(1, 1), (2, 5), (15, 3)])
def test_sine_modes_are_eigenvectors(j, k):
    N = 16
    M, K = fem.assemble(N)
    v = synth.sine_mode_vector(N, j, k)
    lam = _one(N, j) + _one(N, k)
    assert np.linalg.norm(K @ v - lam * (M @ v)) < 1e-11 * lam * np.linalg.norm(M @ v)


def test_full_assembly_invariants():
    N = 12
    kap = synth.grf_kappa(N, 5)
    M, K = fem.assemble_full(N, kap)
    ones = np.ones(M.shape[0])
    assert np.abs(K @ ones).max() < 1e-13 * kap.max()  # constants lie in the Neumann kernel
    assert abs(ones @ M @ ones - 1.0) < 1e-14  # total mass = area of the unit square
    # energy of u = x is int kappa |grad x|^2 = mean of kappa (exact: x is in Q1)
    x = np.tile(np.arange(N + 1) / N, N + 1)
    assert abs(x @ K @ x - kap.mean()) < 1e-13
    y = np.repeat(np.arange(N + 1) / N, N + 1)
    assert abs(y @ K @ y - kap.mean()) < 1e-13
    assert abs(x @ M @ y - 0.25) < 1e-14  # int x*y over the unit square
    assert abs((M - M.T)).max() == 0 and abs((K - K.T)).max() < 1e-16


def test_nine_point_stencils():
    # The 9-point stencils of the interior Q1 operators (a standard derivation from
    # the element matrices) must agree with the assembled CSR at every interior node.
    N = 10
    rng = np.random.default_rng(7)
    kap = rng.uniform(0.3, 3.0, N * N)
    M, K = fem.assemble(N, kap)
    x = rng.standard_normal((N - 1) ** 2)
    X = np.zeros((N + 1, N + 1))
    X[1:N, 1:N] = x.reshape(N - 1, N - 1)
    k2 = kap.reshape(N, N)
    h = 1.0 / N
    Ky = np.zeros((N - 1, N - 1))
    My = np.zeros((N - 1, N - 1))
    for j in range(1, N):
        for i in range(1, N):
            sw, se, nw, ne = k2[j - 1, i - 1], k2[j - 1, i], k2[j, i - 1], k2[j, i]
            c = X[j, i]
            E, W, Nn, S = X[j, i + 1], X[j, i - 1], X[j + 1, i], X[j - 1, i]
            NE, NW, SE, SW = X[j + 1, i + 1], X[j + 1, i - 1], X[j - 1, i + 1], X[j - 1, i - 1]
            Ky[j - 1, i - 1] = (2 / 3) * (sw + se + ne + nw) * c - (1 / 6) * (
                (ne + se) * E + (nw + sw) * W + (ne + nw) * Nn + (se + sw) * S
            ) - (1 / 3) * (ne * NE + nw * NW + se * SE + sw * SW)
            My[j - 1, i - 1] = h * h / 36 * (16 * c + 4 * (E + W + Nn + S) + (NE + NW + SE + SW))
    assert np.abs(K @ x - Ky.ravel()).max() < 1e-13
    assert np.abs(M @ x - My.ravel()).max() < 1e-17


def test_element_gather_roundtrip():
    N = 6
    v = np.arange(1, (N - 1) ** 2 + 1, dtype=float)
    g = fem.element_gather(N, v)
    # element (1,1): nodes (1,1),(2,1),(2,2),(1,2) -> dofs 0,1,6,5 (1-based values 1,2,7,6)
    assert list(g[1 * N + 1]) == [1.0, 2.0, 7.0, 6.0]
    # element (0,0) touches only node (1,1) in its (1,1) corner
    assert list(g[0]) == [0.0, 0.0, 1.0, 0.0]
