"""Butcher tableaux for the stepper (product side).

Radau IIA(s) and Gauss-Legendre(s) are collocation methods (Appendix A): given
the abscissae c, the weights b and the matrix A follow from the simplifying
conditions B(s) and C(s) of the collocation construction,
    sum_j b_j c_j^{k-1} = 1/k,   sum_j a_ij c_j^{k-1} = c_i^k / k,   k = 1..s,
which are s x s Vandermonde systems solved here directly. Abscissae: Radau IIA
uses the right Radau points, the zeros of P_s(2x-1) - P_{s-1}(2x-1); Gauss uses
the zeros of P_s(2x-1) (P_k the Legendre polynomials). The DIRK tableaux of
Appendix A are given by their printed definitions (Alexander's z formula read
with the exponent 2; WSODIRK433 with a_31 = -1.08354073).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg


def _from_nodes(c, name):
    c = np.asarray(c, dtype=np.float64)
    s = c.size
    Vt = np.vander(c, s, increasing=True).T  # Vt[k, j] = c_j^k
    k = np.arange(1, s + 1)
    b = np.linalg.solve(Vt, 1.0 / k)
    A = np.linalg.solve(Vt, (c[None, :] ** k[:, None] / k[:, None])).T
    return {"A": A, "b": b, "c": c, "name": name}


def radau_iia(s: int) -> dict:
    if s == 1:
        return {"A": np.array([[1.0]]), "b": np.array([1.0]), "c": np.array([1.0]), "name": "RadauIIA(1)"}
    ps = np.zeros(s + 1)
    ps[s] = 1.0
    ps[s - 1] = -1.0
    x = np.sort(leg.legroots(ps).real)
    c = (x + 1.0) / 2.0
    c[-1] = 1.0
    return _from_nodes(c, f"RadauIIA({s})")


def gauss_legendre(s: int) -> dict:
    x, _ = leg.leggauss(s)
    return _from_nodes((np.sort(x) + 1.0) / 2.0, f"GaussLegendre({s})")


def lobatto_iiic2() -> dict:
    return {"A": np.array([[0.5, -0.5], [0.5, 0.5]]), "b": np.array([0.5, 0.5]), "c": np.array([0.0, 1.0]),
            "name": "LobattoIIIC(2)"}


def alexander() -> dict:
    r = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    r = r[np.abs(r.imag) < 1e-12].real
    x = float(r[(r > 1.0 / 6.0) & (r < 0.5)][0])
    y = -1.5 * x * x + 4.0 * x - 0.25
    z = 1.5 * x * x - 5.0 * x + 1.25
    A = np.array([[x, 0, 0], [(1 - x) / 2, x, 0], [y, z, x]], dtype=np.float64)
    return {"A": A, "b": A[2].copy(), "c": A.sum(1), "name": "Alexander"}


def wsodirk433() -> dict:
    A = np.array([[0.13756544, 0, 0, 0], [0.56695123, 0.23483889, 0, 0], [-1.08354073, 2.96618224, 0.44915522, 0],
                  [0.59761292, -0.43420998, -0.05305815, 0.88965521]], dtype=np.float64)
    return {"A": A, "b": A[3].copy(), "c": np.array([0.13756544, 0.80179012, 2.33179673, 1.0]), "name": "WSODIRK433"}


def by_name(name: str) -> dict:
    name = name.lower()
    for pre, f in (("radauiia", radau_iia), ("radau", radau_iia), ("gausslegendre", gauss_legendre),
                   ("gauss", gauss_legendre), ("gl", gauss_legendre)):
        if name.startswith(pre) and name[len(pre):].strip("()").isdigit():
            return f(int(name[len(pre):].strip("()")))
    return {"lobattoiiic2": lobatto_iiic2, "alexander": alexander, "wsodirk433": wsodirk433}[name]()
