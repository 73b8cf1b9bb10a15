"""Pins of the oracle's 1D rules and Lagrange basis against closed forms."""
import math

import numpy as np
import pytest

from oracle.basis import gauss_legendre, gauss_lobatto_nodes, lagrange_derivatives


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exact_up_to_degree_2n_minus_1(n):
    x, w = gauss_legendre(n)
    for m in range(2 * n):
        assert abs(np.dot(w, x**m) - 1.0 / (m + 1)) < 1e-15 * (m + 1) + 2e-16
    # degree 2n is not: the error is (n!)^4 / ((2n+1) ((2n)!)^2) on [0, 1]
    err = math.factorial(n) ** 4 / ((2 * n + 1) * math.factorial(2 * n) ** 2)
    if err > 1e-11:
        assert abs((1.0 / (2 * n + 1) - np.dot(w, x ** (2 * n))) / err - 1.0) < 1e-4


def test_gauss_lobatto_closed_forms():
    assert np.allclose(gauss_lobatto_nodes(2), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(gauss_lobatto_nodes(3), [0.0, 0.5, 1.0], atol=1e-16)
    s5 = math.sqrt(5.0) / 10.0
    assert np.allclose(gauss_lobatto_nodes(4), [0.0, 0.5 - s5, 0.5 + s5, 1.0], atol=1e-15)
    s = 0.5 * math.sqrt(3.0 / 7.0)
    assert np.allclose(gauss_lobatto_nodes(5), [0.0, 0.5 - s, 0.5, 0.5 + s, 1.0], atol=1e-15)


@pytest.mark.parametrize("n", range(2, 9))
def test_gauss_lobatto_rule_exactness(n):
    # with its own weights the Lobatto rule integrates degree 2n-3 exactly;
    # weights from the Lagrange basis integrated exactly by Gauss
    xl = gauss_lobatto_nodes(n)
    xg, wg = gauss_legendre(n)
    L = lagrange_derivatives(xl, xg, 0)[0]
    wl = wg @ L
    for m in range(2 * n - 2):
        assert abs(np.dot(wl, xl**m) - 1.0 / (m + 1)) < 1e-13


@pytest.mark.parametrize("n", range(2, 9))
def test_lagrange_interpolates_monomials_and_derivatives(n):
    nodes = gauss_lobatto_nodes(n)
    pts = np.array([0.0, 0.13, 0.5, 0.77, 1.0])
    D = lagrange_derivatives(nodes, pts, n - 1)
    # delta property
    assert np.allclose(lagrange_derivatives(nodes, nodes, 0)[0], np.eye(n), atol=1e-14)
    for m in range(n):
        coeffs = nodes**m
        for r in range(n):
            exact = math.factorial(m) / math.factorial(m - r) * pts ** (m - r) if r <= m else 0 * pts
            got = D[r] @ coeffs
            assert np.allclose(got, exact, atol=1e-10 * max(1, n**r), rtol=1e-11), (m, r)
