"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random numbers and samples fields on the grid; it holds
none of the time-stepping arithmetic. Everything returned here is an *input*
(initial data, a diffusivity field, finite-difference directions), so both the
CPU oracle and the GPU library consume identical bytes.

Layouts (all NumPy float64, C order):
  * nodal vectors: the (N-1)^2 interior nodes of the uniform N x N grid on the
    unit square, row-major by y with x fastest: node (i, j) (x = i/N, y = j/N,
    1 <= i, j <= N-1) sits at index (j-1)*(N-1) + (i-1).
  * element fields: N x N, element (ex, ey) covering [ex/N, (ex+1)/N] x
    [ey/N, (ey+1)/N] sits at index ey*N + ex.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "interior_coords",
    "sine_mode_amplitudes",
    "sine_modes_u0",
    "sine_mode_vector",
    "white_noise_u0",
    "grf_log_kappa",
    "grf_kappa",
    "random_directions",
    "random_stage_block",
    "sample_indices",
    "sketch_vectors",
]


def interior_coords(N: int):
    """Return (x, y) coordinates of the interior nodes in the nodal layout."""
    t = np.arange(1, N, dtype=np.float64) / N
    X, Y = np.meshgrid(t, t, indexing="xy")  # Y varies along rows, X along columns
    return X.ravel(), Y.ravel()


def sine_mode_vector(N: int, j: int, k: int) -> np.ndarray:
    """Nodal interpolant of sin(j*pi*x) * sin(k*pi*y) on the interior nodes."""
    x, y = interior_coords(N)
    return np.sin(j * np.pi * x) * np.sin(k * np.pi * y)


def sine_mode_amplitudes(seed: int = 0, modes: int = 4) -> np.ndarray:
    """N(0,1) amplitudes alpha[j-1, k-1] for the modes (j, k) in {1..modes}^2.

    Drawn from numpy.random.default_rng(seed) in row-major (j, k) order.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((modes, modes))


def sine_modes_u0(N: int, seed: int = 0, modes: int = 4):
    """Initial data: a seeded sum of modes*modes sine modes with N(0,1) amplitudes.

    Returns (u0, amplitudes) where u0 = sum_{j,k} alpha[j-1,k-1] sin(j pi x) sin(k pi y)
    interpolated at the interior nodes.
    """
    amps = sine_mode_amplitudes(seed, modes)
    x, y = interior_coords(N)
    u = np.zeros_like(x)
    for j in range(1, modes + 1):
        sx = np.sin(j * np.pi * x)
        for k in range(1, modes + 1):
            u += amps[j - 1, k - 1] * sx * np.sin(k * np.pi * y)
    return u, amps


def white_noise_u0(N: int, seed: int = 4) -> np.ndarray:
    """White-noise interior nodal vector (stress input for iteration counts)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N - 1) * (N - 1))


def grf_log_kappa(N: int, seed: int, corr_len: float = 0.1, std: float = 1.0) -> np.ndarray:
    """Gaussian random field g on the N x N element centres.

    Squared-exponential covariance std^2 * exp(-r^2 / (2 corr_len^2)), sampled
    exactly by circulant embedding on a 2N x 2N periodic grid of side 2 (the
    wrap-around error is exp(-(1/corr_len)^2 / 2), negligible for corr_len 0.1)
    and cropped to the unit square. Returns an (N*N,) array, element layout.
    """
    h = 1.0 / N
    P = 2 * N
    m = np.arange(P)
    d = np.minimum(m, P - m) * h
    D1, D2 = np.meshgrid(d, d, indexing="ij")
    c = std * std * np.exp(-(D1 * D1 + D2 * D2) / (2.0 * corr_len * corr_len))
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    z = np.fft.fft2(np.sqrt(lam / (P * P)) * xi)
    g = z.real[:N, :N]
    return np.ascontiguousarray(g).ravel()


def grf_kappa(N: int, seed: int, corr_len: float = 0.1, std: float = 1.0) -> np.ndarray:
    """Per-element diffusivity kappa = exp(g), g from :func:`grf_log_kappa`."""
    return np.exp(grf_log_kappa(N, seed, corr_len, std))


def random_directions(count: int, dim: int, seed: int = 3) -> np.ndarray:
    """`count` unit vectors d ~ N(0, I)/|.|, shape (count, dim)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, dim))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_stage_block(N: int, s: int, seed: int) -> np.ndarray:
    """Random s x (N-1)^2 block (stage-major), uniform in [-1, 1)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(s, (N - 1) * (N - 1)))


def sample_indices(n: int, count: int = 4096, seed: int = 12345) -> np.ndarray:
    """Sorted seeded sample of `count` distinct indices in [0, n) (full-size parity spot checks)."""
    return np.sort(np.random.default_rng(seed).choice(n, size=min(count, n), replace=False))


def sketch_vectors(n: int, count: int = 8, seed: int = 54321) -> np.ndarray:
    """`count` seeded N(0, I) vectors of length n; projections onto them sketch a vector's error."""
    return np.random.default_rng(seed).standard_normal((count, n))
