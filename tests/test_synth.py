"""Checks of the seeded input generators."""
import numpy as np

import synth


def test_deterministic_and_shapes():
    a1, _ = synth.sine_modes_u0(32, 0)
    a2, amps = synth.sine_modes_u0(32, 0)
    assert a1.shape == (31 * 31,) and np.array_equal(a1, a2) and amps.shape == (4, 4)
    k1 = synth.grf_kappa(16, 1)
    assert k1.shape == (256,) and np.array_equal(k1, synth.grf_kappa(16, 1))
    assert not np.array_equal(k1, synth.grf_kappa(16, 2))
    assert np.all(k1 > 0)


def test_sine_mode_layout():
    N = 8
    v = synth.sine_mode_vector(N, 1, 2).reshape(N - 1, N - 1)  # rows = y
    assert abs(v[0, 3] - np.sin(np.pi * 4 / 8) * np.sin(2 * np.pi * 1 / 8)) < 1e-15


def test_grf_statistics():
    g = np.stack([synth.grf_log_kappa(64, s) for s in range(20)])
    assert 0.8 < g.var() < 1.2  # unit variance
    assert abs(g.mean()) < 0.2
    # correlation at a lag of one correlation length (0.1 = 6.4 elements at N = 64): exp(-1/2)
    G = g.reshape(20, 64, 64)
    c = np.mean(G[:, :, :-6] * G[:, :, 6:]) / g.var()
    assert abs(c - np.exp(-0.5 * (6 / 6.4) ** 2)) < 0.12


def test_directions_unit():
    d = synth.random_directions(32, 100, seed=3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
