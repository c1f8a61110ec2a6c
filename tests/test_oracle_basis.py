"""Pins of the oracle's nodal basis (Sec. 2.6: nodal DGSEM on Gauss points).

Each check compares with something the oracle does not compute itself: the
library Gauss rule, exact polynomial calculus, and the summation-by-parts
identity that integration by parts imposes on any Gauss collocation basis.
"""
import numpy as np
import pytest

from oracle.basis import Basis, legendre


@pytest.mark.parametrize("P", range(1, 11))
def test_gauss_nodes_match_library(P):
    b = Basis(P)
    x, w = np.polynomial.legendre.leggauss(P + 1)
    assert np.max(np.abs(b.nodes - x)) < 1e-15
    assert np.max(np.abs(b.weights - w)) < 1e-14


@pytest.mark.parametrize("P", [1, 2, 3, 5, 6, 8])
def test_derivative_matrix_exact_to_degree_P(P):
    b = Basis(P)
    scale = np.max(np.abs(b.D))
    for m in range(P + 1):
        exact = m * b.nodes ** (m - 1) if m > 0 else np.zeros_like(b.nodes)
        assert np.max(np.abs(b.D @ b.nodes ** m - exact)) < 2e-14 * scale * max(1, m)
    # degree P+1 is not representable on P+1 points
    m = P + 1
    assert np.max(np.abs(b.D @ b.nodes ** m - m * b.nodes ** (m - 1))) > 1e-6


@pytest.mark.parametrize("P", [1, 3, 6, 8])
def test_boundary_interpolation_exact(P):
    b = Basis(P)
    for m in range(P + 1):
        assert abs(b.bp @ b.nodes ** m - 1.0) < 1e-13
        assert abs(b.bm @ b.nodes ** m - (-1.0) ** m) < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 6, 8])
def test_summation_by_parts(P):
    """W D + D^T W = b+ b+^T - b- b-^T (discrete integration by parts)."""
    b = Basis(P)
    W = np.diag(b.weights)
    lhs = W @ b.D + b.D.T @ W
    rhs = np.outer(b.bp, b.bp) - np.outer(b.bm, b.bm)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(b.D))


def test_legendre_against_numpy():
    x = np.linspace(-1, 1, 37)
    for n in range(9):
        c = np.zeros(n + 1)
        c[n] = 1
        val, der = legendre(n, x)
        assert np.max(np.abs(val - np.polynomial.legendre.legval(x, c))) < 1e-14
        assert np.max(np.abs(der - np.polynomial.legendre.legval(x, np.polynomial.legendre.legder(c)))) < 1e-12
