"""Pins of the oracle's global operator: brute-force assembly, closed forms, eigenvalues."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, mesh


def _nodal(d, k, level, f1d):
    n = mesh.n1d(k, level)
    h = mesh.mesh_size(level)
    g = basis.gll_nodes(k)
    xs = np.concatenate([c * h + g[:-1] * h for c in range(2 ** level)] + [[1.0]])
    U = np.ones((1,) * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n
        U = U * f1d(xs).reshape(shape)
    return U.reshape(-1)


@pytest.mark.parametrize("d,k,level", [(2, 1, 2), (2, 2, 2), (2, 3, 1), (3, 1, 2), (3, 2, 1)])
def test_kronecker_operator_equals_cell_assembly(d, k, level):
    A = mesh.operator_matrix(d, k, level).toarray()
    B = mesh.assembled_matrix_bruteforce(d, k, level)
    inner = mesh.interior_ids(d, k, level)
    assert np.allclose(A, B[np.ix_(inner, inner)], atol=1e-12)


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (3, 2, 2), (2, 5, 2)])
def test_axiswise_apply_equals_matrix(d, k, level):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(mesh.n1d(k, level) ** d)
    inner = mesh.interior_ids(d, k, level)
    y = mesh.apply_operator(d, k, level, x)
    A = mesh.operator_matrix(d, k, level)
    assert np.allclose(y[inner], A @ x[inner], atol=1e-12)
    assert np.all(y[mesh.boundary_mask(d, k, level)] == 0)


@pytest.mark.parametrize("d,k,level", [(2, 2, 1), (2, 2, 3), (2, 4, 2), (3, 2, 2), (3, 3, 1), (3, 4, 1)])
def test_bubble_energy(d, k, level):
    """u = prod x_a(1-x_a) lies in Q_k (k >= 2): x^T A x = |u|_{H1}^2 = 1/45 (2D), 1/900 (3D)."""
    u = _nodal(d, k, level, lambda x: x * (1 - x))
    e = u @ mesh.apply_operator(d, k, level, u)
    assert abs(e - (1 / 45 if d == 2 else 1 / 900)) < 1e-14


@pytest.mark.parametrize("level", [2, 3, 4])
def test_q1_diagonal(level):
    A2 = mesh.operator_matrix(2, 1, level)
    assert np.allclose(A2.diagonal(), 8 / 3)
    h = mesh.mesh_size(level)
    A3 = mesh.operator_matrix(3, 1, level)
    assert np.allclose(A3.diagonal(), 8 * h / 3)


@pytest.mark.parametrize("level", [2, 3])
def test_q1_generalised_eigenvalues_closed_form(level):
    """1D Q1: lambda_j = (6/h^2)(1 - cos j pi h)/(2 + cos j pi h); 2D eigenvalues are pairwise sums."""
    h = mesh.mesh_size(level)
    A1, M1 = mesh.global_1d_matrices(1, level)
    inner = slice(1, mesh.n1d(1, level) - 1)
    A1 = A1[inner, inner].toarray()
    M1 = M1[inner, inner].toarray()
    j = np.arange(1, 2 ** level)
    lam = 6 / h ** 2 * (1 - np.cos(j * math.pi * h)) / (2 + np.cos(j * math.pi * h))
    assert np.allclose(np.sort(sla.eigh(A1, M1, eigvals_only=True)), np.sort(lam), rtol=1e-12)
    A = mesh.operator_matrix(2, 1, level).toarray()
    ev = sla.eigh(A, np.kron(M1, M1), eigvals_only=True)
    assert np.allclose(np.sort(ev), np.sort((lam[:, None] + lam[None, :]).reshape(-1)), rtol=1e-10)


@pytest.mark.parametrize("d,k,level", [(2, 3, 2), (3, 2, 2)])
def test_operator_spd(d, k, level):
    A = mesh.operator_matrix(d, k, level).toarray()
    assert np.allclose(A, A.T, atol=1e-14)
    sla.cholesky(A)


@pytest.mark.parametrize("d,k,L", [(2, 1, 3), (2, 4, 2), (2, 7, 2), (3, 1, 2), (3, 3, 2), (3, 5, 1)])
def test_operator_rows_equal_the_full_apply(d, k, L):
    """Rows computed one at a time from the node's stencil box equal the axis-wise apply, including
    rows next to and on the Dirichlet boundary (boundary values of x poisoned: never read)."""
    import synth
    x = synth.random_interior(d, k, L, 13)
    ref = mesh.apply_operator(d, k, L, x)
    xg = x.copy()
    xg[mesh.boundary_mask(d, k, L)] = np.nan
    n = mesh.n1d(k, L)
    coords = np.array(list(np.ndindex(*([n] * d))))[:, ::-1]  # (c_0, ..., c_{d-1}) in flat order
    got = mesh.operator_rows(d, k, L, coords, xg)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,k,L", [(2, 2, 2), (3, 1, 2), (3, 2, 1)])
def test_absolute_operator_rows_equal_the_explicit_kronecker_sum(d, k, L):
    """The magnitude sum used for tolerances on computed rows, sum_dir ((x)_a |A1 or M1|) |x|, equals
    the same sum formed from explicit Kronecker products of the dense interior 1D matrices; it also
    bounds |A x| entrywise."""
    import synth
    x = synth.random_interior(d, k, L, 17)
    n = mesh.n1d(k, L)
    A1, M1 = (abs(m.toarray()) for m in mesh.global_1d_matrices(k, L))
    inner = np.arange(1, n - 1)
    A1, M1 = A1[np.ix_(inner, inner)], M1[np.ix_(inner, inner)]
    big = 0.0
    for direction in range(d):
        term = np.ones((1, 1))
        for a in reversed(range(d)):  # leftmost factor = slowest axis
            term = np.kron(term, A1 if a == direction else M1)
        big = big + term
    ids = mesh.interior_ids(d, k, L)
    ref = big @ np.abs(x[ids])
    coords = np.array(list(np.ndindex(*([n] * d))))[:, ::-1]
    got = mesh.operator_rows(d, k, L, coords, x, absolute=True)
    assert np.max(np.abs(got[ids] - ref)) <= 1e-14 * np.max(ref)
    assert np.all(got[mesh.boundary_mask(d, k, L)] == 0.0)
    assert np.all(np.abs(mesh.apply_operator(d, k, L, x)) <= got * (1 + 1e-14))
