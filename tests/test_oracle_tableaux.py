"""Pins for oracle.tableaux: printed tableaux, order conditions, Pade forms."""
import numpy as np
import pytest

from oracle import tableaux as T


@pytest.mark.parametrize("s", [1, 2, 3])
def test_radau_collocation_matches_printed(s):
    # Appendix A prints Radau IIA(1..3); the collocation recipe must reproduce them
    a, p = T.radau_iia(s), T.radau_iia_printed(s)
    for key in ("A", "b", "c"):
        assert np.abs(a[key] - p[key]).max() < 1e-14


@pytest.mark.parametrize("make,s", [(T.radau_iia, 1), (T.radau_iia, 2), (T.radau_iia, 3), (T.radau_iia, 4),
                                    (T.gauss_legendre, 1), (T.gauss_legendre, 2), (T.gauss_legendre, 3),
                                    (T.gauss_legendre, 4)])
def test_collocation_order_conditions(make, s):
    tab = make(s)
    A, b, c = tab["A"], tab["b"], tab["c"]
    # quadrature order: 2s for Gauss, 2s-1 for Radau
    q = 2 * s if make is T.gauss_legendre else 2 * s - 1
    for k in range(1, q + 1):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-13
    # stage order s: sum_j a_ij c_j^{k-1} = c_i^k / k
    for k in range(1, s + 1):
        assert np.abs(A @ c ** (k - 1) - c**k / k).max() < 1e-13
    if make is T.radau_iia:
        assert abs(c[-1] - 1.0) < 1e-15
        assert np.abs(A[-1] - b).max() < 1e-14  # stiffly accurate


def test_gauss2_nodes_closed_form():
    c = T.gauss_legendre(2)["c"]
    assert np.abs(c - np.array([0.5 - np.sqrt(3) / 6, 0.5 + np.sqrt(3) / 6])).max() < 1e-15


def _pade(z, num, den):
    return np.polyval(num[::-1], z) / np.polyval(den[::-1], z)


@pytest.mark.parametrize("z", [-0.5, -7.0, -300.0, 0.3 + 0.2j])
def test_stability_function_pade(z):
    # Hairer & Wanner: Radau IIA(s) -> (s-1, s) Pade; Gauss(s) -> (s, s) Pade; Lobatto IIIC(2) -> (0, 2)
    R2 = T.stability_function(T.radau_iia(2), z)[0]
    assert abs(R2 - _pade(z, [1, 1 / 3], [1, -2 / 3, 1 / 6])) < 1e-13 * max(1, abs(R2))
    R3 = T.stability_function(T.radau_iia(3), z)[0]
    assert abs(R3 - _pade(z, [1, 2 / 5, 1 / 20], [1, -3 / 5, 3 / 20, -1 / 60])) < 1e-13
    G4 = T.stability_function(T.gauss_legendre(4), z)[0]
    P = [1, 1 / 2, 3 / 28, 1 / 84, 1 / 1680]
    assert abs(G4 - _pade(z, P, [p * (-1) ** i for i, p in enumerate(P)])) < 1e-12
    L2 = T.stability_function(T.lobatto_iiic2(), z)[0]
    assert abs(L2 - 1.0 / (1 - z + z * z / 2)) < 1e-13


def test_gauss4_not_l_stable():
    R = T.stability_function(T.gauss_legendre(4), -1e8)[0].real
    assert 0.9999 < R < 1.0


def test_alexander_order3_and_l_stable():
    tab = T.alexander()
    A, b, c = tab["A"], tab["b"], tab["c"]
    x = A[0, 0]
    assert abs(x**3 - 3 * x**2 + 1.5 * x - 1 / 6) < 1e-14 and 1 / 6 < x < 0.5
    assert np.abs(A.sum(1) - c).max() < 1e-14
    assert abs(b.sum() - 1) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ c**2 - 1 / 3) < 1e-14
    assert abs(b @ A @ c - 1 / 6) < 1e-14
    assert abs(T.stability_function(tab, -1e12)[0]) < 1e-9
    # x (the root of the cubic above in (1/6, 1/2)) and the last row of A, to ten digits
    assert abs(x - 0.4358665215) < 1e-10 and abs(A[2, 0] - 1.2084966492) < 1e-9
    assert abs(A[2, 1] + 0.6443631707) < 1e-9


def test_wsodirk433_reading():
    tab = T.wsodirk433()
    A, b, c = tab["A"], tab["b"], tab["c"]
    assert np.abs(A.sum(1) - c).max() < 2e-8  # row sums reproduce the printed c (8 digits)
    assert abs(b.sum() - 1) < 1e-7
    assert abs(b @ c - 0.5) < 1e-7
    assert abs(b @ c**2 - 1 / 3) < 1e-7
    assert abs(b @ A @ c - 1 / 6) < 1e-7
