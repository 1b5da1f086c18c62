"""Pins of the oracle's prolongation (embedding) and restriction (transpose), Sec. 2.1."""
import numpy as np
import pytest

from oracle import basis, mesh, transfer


def test_q1_prolongation_stencil():
    P1 = transfer.prolongation_1d(1, 2)  # 5 fine nodes from 3 coarse nodes
    assert np.allclose(P1, [[1, 0, 0], [.5, .5, 0], [0, 1, 0], [0, .5, .5], [0, 0, 1]])


def _nodal(d, k, level, fs):
    n = mesh.n1d(k, level)
    h = mesh.mesh_size(level)
    g = basis.gll_nodes(k)
    xs = np.concatenate([c * h + g[:-1] * h for c in range(2 ** level)] + [[1.0]])
    U = np.ones((1,) * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n
        U = U * fs[a](xs).reshape(shape)
    return U.reshape(-1)


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (2, 4, 2), (3, 3, 2), (2, 7, 2)])
def test_prolongation_reproduces_coarse_polynomials(d, k, level):
    """A polynomial of degree <= k per axis vanishing on the boundary is embedded exactly."""
    rng = np.random.default_rng(0)
    fs = []
    for a in range(d):
        c = rng.standard_normal(k - 1)
        fs.append(lambda x, c=c: x * (1 - x) * np.polyval(c, x))
    ec = _nodal(d, k, level - 1, fs)
    ef = _nodal(d, k, level, fs)
    assert np.allclose(transfer.prolongate(d, k, level, ec), ef, atol=1e-13)


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (3, 2, 2), (2, 3, 2), (2, 1, 4)])
def test_galerkin_identity(d, k, level):
    """P^T A_l P = A_{l-1}: nested spaces and the embedding as prolongation."""
    nf, nc = mesh.n1d(k, level), mesh.n1d(k, level - 1)
    inner_c = mesh.interior_ids(d, k, level - 1)
    cols = []
    for j in inner_c:
        e = np.zeros(nc ** d)
        e[j] = 1
        cols.append(transfer.prolongate(d, k, level, e))
    P = np.array(cols).T
    Af = mesh.operator_matrix(d, k, level).toarray()
    inner_f = mesh.interior_ids(d, k, level)
    Pi = P[inner_f]
    Ac = mesh.operator_matrix(d, k, level - 1).toarray()
    assert np.allclose(Pi.T @ Af @ Pi, Ac, atol=1e-12 * np.abs(Ac).max())


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (3, 2, 2)])
def test_restriction_is_dense_transpose(d, k, level):
    rng = np.random.default_rng(1)
    nf, nc = mesh.n1d(k, level), mesh.n1d(k, level - 1)
    r = rng.standard_normal(nf ** d)
    r[mesh.boundary_mask(d, k, level)] = 0
    P = np.zeros((nf ** d, nc ** d))
    for j in mesh.interior_ids(d, k, level - 1):
        e = np.zeros(nc ** d)
        e[j] = 1
        P[:, j] = transfer.prolongate(d, k, level, e)
    assert np.allclose(transfer.restrict(d, k, level, r), P.T @ r, atol=1e-13)
