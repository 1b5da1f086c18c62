"""Pins of the oracle's 1D building blocks against closed forms and independent quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import basis


def test_gll_nodes_closed_forms():
    assert np.allclose(basis.gll_nodes(1), [0, 1], atol=0, rtol=0)
    assert np.allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    a = 1 / math.sqrt(5)
    assert np.allclose(basis.gll_nodes(3), [0, (1 - a) / 2, (1 + a) / 2, 1], atol=1e-15)
    b = math.sqrt(3 / 7)
    assert np.allclose(basis.gll_nodes(4), [0, (1 - b) / 2, 0.5, (1 + b) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("k", range(1, 9))
def test_gll_nodes_symmetric_and_sorted(k):
    g = basis.gll_nodes(k)
    assert len(g) == k + 1
    assert np.all(np.diff(g) > 0)
    assert np.allclose(g + g[::-1], 1.0, atol=1e-14)


@pytest.mark.parametrize("nq", range(1, 9))
def test_gauss_rule_exact_for_monomials(nq):
    x, w = basis.gauss_rule(nq)
    for p in range(2 * nq):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14


@pytest.mark.parametrize("k", range(1, 8))
def test_lagrange_basis_properties(k):
    g = basis.gll_nodes(k)
    assert np.allclose(basis.lagrange_values(g, g), np.eye(k + 1), atol=1e-13)
    xs = np.linspace(0, 1, 17)
    assert np.allclose(basis.lagrange_values(g, xs).sum(0), 1.0, atol=1e-12)
    assert np.allclose(basis.lagrange_derivatives(g, xs).sum(0), 0.0, atol=1e-10)
    # derivative against a central difference
    e = 1e-6
    fd = (basis.lagrange_values(g, xs[1:-1] + e) - basis.lagrange_values(g, xs[1:-1] - e)) / (2 * e)
    assert np.allclose(basis.lagrange_derivatives(g, xs[1:-1]), fd, atol=1e-6 * k ** 3)


def test_reference_matrices_closed_forms():
    A, M = basis.reference_matrices(1)
    assert np.allclose(A, [[1, -1], [-1, 1]], atol=1e-15)
    assert np.allclose(M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    A, M = basis.reference_matrices(2)
    assert np.allclose(A, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3, atol=1e-14)
    assert np.allclose(M, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30, atol=1e-15)


@pytest.mark.parametrize("k", range(1, 8))
def test_reference_matrices_invariants(k):
    A, M = basis.reference_matrices(k)
    one = np.ones(k + 1)
    assert np.allclose(A @ one, 0, atol=1e-11)
    assert abs(one @ M @ one - 1.0) < 1e-14
    assert np.allclose(A, A.T) and np.allclose(M, M.T)
    assert np.all(np.linalg.eigvalsh(M) > 0)
    # x^T A x for the nodal values of x -> x is int (1)^2 = 1
    g = basis.gll_nodes(k)
    assert abs(g @ A @ g - 1.0) < 1e-11


@pytest.mark.parametrize("k", [2, 3])
def test_reference_matrices_against_adaptive_quadrature(k):
    """Entries by scipy's adaptive quadrature of the explicit Lagrange polynomials."""
    g = basis.gll_nodes(k)
    A, M = basis.reference_matrices(k)

    def phi(i, x):
        return np.prod([(x - g[j]) / (g[i] - g[j]) for j in range(k + 1) if j != i])

    def dphi(i, x, e=1e-6):
        return (phi(i, x + e) - phi(i, x - e)) / (2 * e)

    for i in range(k + 1):
        for j in range(k + 1):
            m, _ = integrate.quad(lambda x: phi(i, x) * phi(j, x), 0, 1, epsabs=1e-14)
            a, _ = integrate.quad(lambda x: dphi(i, x) * dphi(j, x), 0, 1, epsabs=1e-12)
            assert abs(M[i, j] - m) < 1e-13
            assert abs(A[i, j] - a) < 1e-6


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_cell_matrix_kronecker_equals_pointwise_quadrature(d, k):
    h = 0.25
    assert np.allclose(basis.cell_matrix(d, k, h), basis.cell_matrix_bruteforce(d, k, h), atol=1e-13)
