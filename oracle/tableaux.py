"""Butcher tableaux for the oracle (FP64, CPU).

Test infrastructure only (see the package docstring).

A tableau is a dict with keys "A" (s x s), "b" (s,), "c" (s,), "name".
Sources:
  * Radau IIA(s): the collocation recipe of Appendix A -- the abscissae c_i are
    the roots of d^{s-1}/dx^{s-1}[x^{s-1}(x-1)^s]; then a_ij and b_j are the
    integrals of the Lagrange basis polynomials on the c's (the usual
    collocation construction): a_ij = int_0^{c_i} l_j, b_j = int_0^1 l_j.
  * Gauss-Legendre(s): the paper does not print it; the same collocation
    construction on the roots of the shifted Legendre polynomial P_s(2x-1).
  * Printed tableaux of Appendix A (Radau IIA 1-3, Alexander's DIRK,
    WSODIRK433) and the two-stage Lobatto IIIC of Section 2 (eq:lobattotableau),
    with the two printing defects read as follows:
      - Alexander: the z formula lost an exponent; it is read as
        z = 3/2 x^2 - 5 x + 5/4 (the order-3 conditions then hold);
      - WSODIRK433: the first entry of row 3 is read as -1.08354073 (the row
        sum then equals c_3 = 2.33179673).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre as L


def _collocation(c: np.ndarray, name: str) -> dict:
    """Collocation tableau on the abscissae c: integrate the Lagrange basis."""
    c = np.asarray(c, dtype=np.float64)
    s = c.size
    A = np.zeros((s, s))
    b = np.zeros(s)
    for j in range(s):
        lj = Polynomial([1.0])
        for m in range(s):
            if m != j:
                lj = lj * Polynomial([-c[m], 1.0]) / (c[j] - c[m])
        Ij = lj.integ()  # antiderivative vanishing at 0
        b[j] = Ij(1.0) - Ij(0.0)
        for i in range(s):
            A[i, j] = Ij(c[i]) - Ij(0.0)
    return {"A": A, "b": b, "c": c.copy(), "name": name}


def radau_iia(s: int) -> dict:
    """Radau IIA(s) by the collocation recipe of Appendix A."""
    x_m1 = Polynomial([0.0, 1.0]) ** (s - 1)
    x1 = Polynomial([-1.0, 1.0]) ** s
    p = (x_m1 * x1).deriv(s - 1) if s > 1 else x_m1 * x1
    r = np.sort(p.roots().real)
    # the recipe always yields c_s = 1; snap the root that rounding moved
    r[-1] = 1.0
    return _collocation(r, f"RadauIIA({s})")


def gauss_legendre(s: int) -> dict:
    """Gauss-Legendre(s) collocation tableau (abscissae: roots of P_s(2x-1))."""
    coef = np.zeros(s + 1)
    coef[s] = 1.0
    x = np.sort(L.legroots(coef))
    return _collocation((x + 1.0) / 2.0, f"GaussLegendre({s})")


def radau_iia_printed(s: int) -> dict:
    """Radau IIA(1..3) exactly as printed in Appendix A."""
    if s == 1:
        return {"A": np.array([[1.0]]), "b": np.array([1.0]), "c": np.array([1.0]), "name": "RadauIIA(1) printed"}
    if s == 2:
        A = np.array([[5.0 / 12.0, -1.0 / 12.0], [3.0 / 4.0, 1.0 / 4.0]])
        return {"A": A, "b": np.array([0.75, 0.25]), "c": np.array([1.0 / 3.0, 1.0]), "name": "RadauIIA(2) printed"}
    if s == 3:
        r6 = np.sqrt(6.0)
        A = np.array(
            [
                [11.0 / 45.0 - 7.0 * r6 / 360.0, 37.0 / 225.0 - 169.0 * r6 / 1800.0, -2.0 / 225.0 + r6 / 75.0],
                [37.0 / 225.0 + 169.0 * r6 / 1800.0, 11.0 / 45.0 + 7.0 * r6 / 360.0, -2.0 / 225.0 - r6 / 75.0],
                [4.0 / 9.0 - r6 / 36.0, 4.0 / 9.0 + r6 / 36.0, 1.0 / 9.0],
            ]
        )
        c = np.array([2.0 / 5.0 - r6 / 10.0, 2.0 / 5.0 + r6 / 10.0, 1.0])
        return {"A": A, "b": A[2].copy(), "c": c, "name": "RadauIIA(3) printed"}
    raise ValueError("only s = 1, 2, 3 are printed")


def lobatto_iiic2() -> dict:
    """Two-stage Lobatto IIIC (Section 2, eq:lobattotableau)."""
    A = np.array([[0.5, -0.5], [0.5, 0.5]])
    return {"A": A, "b": np.array([0.5, 0.5]), "c": np.array([0.0, 1.0]), "name": "LobattoIIIC(2)"}


def alexander() -> dict:
    """Alexander's three-stage L-stable DIRK (Appendix A).

    x is the root of x^3 - 3x^2 + 3/2 x - 1/6 in (1/6, 1/2); y = -3/2 x^2 + 4x - 1/4;
    z = 3/2 x^2 - 5x + 5/4 (reading of the misprinted exponent).
    """
    roots = Polynomial([-1.0 / 6.0, 1.5, -3.0, 1.0]).roots()
    roots = roots[np.abs(roots.imag) < 1e-12].real
    x = float(roots[(roots > 1.0 / 6.0) & (roots < 0.5)][0])
    y = -1.5 * x * x + 4.0 * x - 0.25
    z = 1.5 * x * x - 5.0 * x + 1.25
    A = np.array([[x, 0.0, 0.0], [(1.0 - x) / 2.0, x, 0.0], [y, z, x]])
    return {"A": A, "b": np.array([y, z, x]), "c": np.array([x, (1.0 + x) / 2.0, 1.0]), "name": "Alexander"}


def wsodirk433() -> dict:
    """Four-stage DIRK with weak stage order 3 (Appendix A, 8 printed digits).

    a_31 is read as -1.08354073 (see the module docstring).
    """
    A = np.array(
        [
            [0.13756544, 0.0, 0.0, 0.0],
            [0.56695123, 0.23483889, 0.0, 0.0],
            [-1.08354073, 2.96618224, 0.44915522, 0.0],
            [0.59761292, -0.43420998, -0.05305815, 0.88965521],
        ]
    )
    c = np.array([0.13756544, 0.80179012, 2.33179673, 1.0])
    return {"A": A, "b": A[3].copy(), "c": c, "name": "WSODIRK433"}


def backward_euler() -> dict:
    return radau_iia_printed(1)


def stability_function(tab: dict, z):
    """R(z) = 1 + z b^T (I - z A)^{-1} 1: the step map of y' = lambda y with z = dt*lambda.

    Follows from the Runge-Kutta step of Section 2 (eq:stageeq and the update
    y^{n+1} = y^n + dt sum_i b_i k_i) applied to the scalar linear test equation.
    """
    A = np.asarray(tab["A"], dtype=np.complex128)
    b = np.asarray(tab["b"], dtype=np.complex128)
    s = b.size
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    out = np.empty(z.shape, dtype=np.complex128)
    one = np.ones(s, dtype=np.complex128)
    for idx, zz in np.ndenumerate(z):
        out[idx] = 1.0 + zz * (b @ np.linalg.solve(np.eye(s) - zz * A, one))
    return out
