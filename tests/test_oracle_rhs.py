"""Pins of the oracle's load vectors and L2 error (eq:matrix-def, Sec. 4.2)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import basis, mesh, rhs
import synth


@pytest.mark.parametrize("d,k,L", [(2, 2, 2), (2, 3, 1), (3, 1, 2)])
def test_separable_load_vector_equals_pointwise_quadrature(d, k, L):
    kap, co = synth.fourier_modes(d, seed=3, n_modes=3, kappa_max=3)

    def f(p):
        return sum(c * np.prod([np.sin(np.pi * kk[a] * p[a]) for a in range(d)]) for kk, c in zip(kap, co))

    assert np.allclose(rhs.rhs_sine_modes(d, k, L, kap, co), rhs.rhs_bruteforce(d, k, L, f), atol=1e-14)


@pytest.mark.parametrize("k", [1, 3])
def test_1d_load_vector_converges_to_exact_integral(k):
    """With many quadrature points the entries approach int sin(pi x) phi_i exactly (scipy quad)."""
    L = 2
    g_hi = rhs.load_vector_1d(k, L, 1, nq=20)
    h = mesh.mesh_size(L)
    nodes = basis.gll_nodes(k)
    for i in range(mesh.n1d(k, L)):
        cells = [c for c in range(2 ** L) if k * c <= i <= k * c + k]
        tot = 0.0
        for c in cells:
            li = i - k * c
            phi = lambda x: basis.lagrange_values(nodes, [(x - c * h) / h])[li, 0]
            tot += integrate.quad(lambda x: np.sin(np.pi * x) * phi(x), c * h, (c + 1) * h, epsabs=1e-15)[0]
        assert abs(g_hi[i] - tot) < 1e-13


def test_l2_error_of_exact_polynomial_is_zero():
    """u = x(1-x)y(1-y) in Q2 has zero interpolation error; with a sine target the error is the closed form."""
    d, k, L = 2, 2, 2
    n = mesh.n1d(k, L)
    x = np.zeros(n ** d)
    e = rhs.l2_error(d, k, L, x, [[1, 1]], [1.0], nq=8)
    assert abs(e - 0.5) < 1e-6  # || sin(pi x) sin(pi y) ||_L2 = 1/2


def test_random_interior_layout():
    v = synth.random_interior(2, 2, 4, 0)
    bm = mesh.boundary_mask(2, 2, 4)
    assert v.shape == (33 * 33,)
    assert np.all(v[bm] == 0) and np.all(np.abs(v[~bm]) <= 1) and np.all(v[~bm] != 0)


@pytest.mark.parametrize("d,k,L", [(2, 3, 3), (3, 2, 2), (3, 5, 1)])
def test_rhs_entries_at_nodes_equal_the_full_vector(d, k, L):
    import synth
    kap, co = synth.fourier_modes(d, seed=4)
    full = rhs.rhs_sine_modes(d, k, L, kap, co)
    n = mesh.n1d(k, L)
    coords = np.array(list(np.ndindex(*([n] * d))))[:, ::-1]
    assert np.max(np.abs(rhs.rhs_sine_modes_at(d, k, L, kap, co, coords) - full)) <= 1e-15 * np.max(np.abs(full))
