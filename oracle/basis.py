"""1D rules and Lagrange polynomials on the reference interval [0, 1].

Test infrastructure only (see the package docstring).

* Gauss-Legendre rule with n points: quadrature of the structured cells and
  faces, k = p + 1 points per direction (Section 3.2, choice n_q = k).
* Gauss-Lobatto nodes: support points of the nodal Lagrange basis, so that a
  face value is read from the cell values directly (Section 3.2, remark after
  the structured face evaluation).
* Lagrange polynomials and all their derivatives at arbitrary points, through
  the Taylor expansion of the product of linear factors at the point.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(n: int):
    """Gauss-Legendre points and weights mapped to [0, 1] (library routine)."""
    t, w = npleg.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def gauss_lobatto_nodes(n: int) -> np.ndarray:
    """Gauss-Lobatto nodes on [0, 1]: the end points and the roots of P'_{n-1}."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs at least 2 nodes")
    if n == 2:
        return np.array([0.0, 1.0])
    dP = npleg.Legendre.basis(n - 1).deriv()
    inner = np.sort(np.real(dP.roots()))
    t = np.concatenate([[-1.0], inner, [1.0]])
    # symmetrise against root-finder noise
    t = 0.5 * (t - t[::-1])
    return 0.5 * (t + 1.0)


def lagrange_derivatives(nodes: np.ndarray, x, max_order: int) -> np.ndarray:
    """Derivatives of order 0..max_order of the Lagrange polynomials on
    ``nodes`` at the points ``x``.

    Returns an array D[order, point, i].  For each point x0 the polynomial
    L_i(x0 + t) = prod_{j != i} (t + x0 - x_j) / (x_i - x_j) is expanded in t by
    multiplying out the linear factors; the coefficient of t^r times r! is the
    r-th derivative at x0.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.zeros((max_order + 1, xs.size, n))
    for i in range(n):
        # coef[:, r] holds the t^r coefficient for every point at once
        coef = np.zeros((xs.size, n))
        coef[:, 0] = 1.0
        deg = 0
        for j in range(n):
            if j == i:
                continue
            a = (xs - nodes[j]) / (nodes[i] - nodes[j])
            b = 1.0 / (nodes[i] - nodes[j])
            # multiply the polynomial coef[:, 0..deg] by (a + b t)
            new = np.zeros_like(coef)
            new[:, : deg + 1] += a[:, None] * coef[:, : deg + 1]
            new[:, 1 : deg + 2] += b * coef[:, : deg + 1]
            coef = new
            deg += 1
        for r in range(min(max_order, n - 1) + 1):
            out[r, :, i] = coef[:, r] * math.factorial(r)
    return out


def lagrange_values(nodes, x) -> np.ndarray:
    return lagrange_derivatives(nodes, x, 0)[0]
