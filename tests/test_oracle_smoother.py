"""Pins of the oracle's patches, colours, local solves and smoothers (Sec. 2.2, Sec. 2.4)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fastdiag, mesh, smoother


def test_colour_sizes_2d_q2_16x16():
    """16x16 cells: 225 interior vertices in colours of 64, 56, 56, 49."""
    sizes = [len(mesh.patches_of_colour(2, 4, c)) for c in range(4)]
    assert sizes == [64, 56, 56, 49]


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (3, 1, 3), (3, 2, 2)])
def test_same_colour_patches_do_not_interact(d, k, level):
    """Within a colour, no patch interior meets another patch's closure (races impossible)."""
    for c in range(2 ** d):
        verts = mesh.patches_of_colour(d, level, c)
        owner = {}
        for j, v in enumerate(verts):
            for i in mesh.patch_interior_ids(d, k, level, v):
                assert i not in owner
                owner[i] = j
        for j, v in enumerate(verts):
            for i in mesh.patch_closure_ids(d, k, level, v):
                assert owner.get(i, j) == j


@pytest.mark.parametrize("d,k,level", [(2, 2, 3), (2, 3, 2), (3, 2, 2), (3, 1, 3)])
def test_patch_matrices_are_global_submatrices(d, k, level):
    """A_j = A[I_j, I_j] for every patch; Abar_j rows = global rows over the closure."""
    Abar, Aj = smoother.patch_matrices(d, k, level)
    sla.cholesky(Aj)  # SPD
    A = mesh.operator_matrix(d, k, level)
    inner = mesh.interior_ids(d, k, level)
    pos = np.full(mesh.n1d(k, level) ** d, -1)
    pos[inner] = np.arange(len(inner))
    bmask = mesh.boundary_mask(d, k, level)
    for v in mesh.patch_vertices(d, level):
        Ag = smoother.patch_matrix_from_global(d, k, level, v)
        assert np.allclose(Ag, Aj, rtol=0, atol=1e-13 * np.abs(Aj).max())
        rows = pos[mesh.patch_interior_ids(d, k, level, v)]
        clos = mesh.patch_closure_ids(d, k, level, v)
        keep = ~bmask[clos]
        sub = A[rows][:, pos[clos[keep]]].toarray()
        assert np.allclose(sub, Abar[:, keep], atol=1e-13 * np.abs(Aj).max())
        # every nonzero of those global rows lies inside the closure
        assert np.isclose(np.abs(A[rows]).sum(), np.abs(sub).sum())


@pytest.mark.parametrize("d,k", [(2, k) for k in range(1, 8)] + [(3, k) for k in range(1, 6)])
def test_fast_diagonalisation_equals_dense_inverse(d, k):
    h = mesh.mesh_size(3)
    _, Aj = smoother.patch_matrices(d, k, 3)
    inv = np.linalg.inv(Aj)
    assert np.abs(fastdiag.inverse(d, k, h) - inv).max() <= 1e-13 * np.abs(inv).max()
    S, lam = fastdiag.eigen_1d(k, h)
    A1, M1 = fastdiag.patch_1d_matrices(k, h)
    assert np.allclose(S.T @ M1 @ S, np.eye(2 * k - 1), atol=1e-12)
    assert np.allclose(A1 @ S, M1 @ S @ np.diag(lam), atol=1e-9 * lam.max())


@pytest.mark.parametrize("d", [2, 3])
def test_q1_patch_solve_is_point_jacobi(d):
    """Q1: one interior node per patch, A_j^{-1} = 1 / diag (Sec. 3.1.1)."""
    level = 3
    r = np.random.default_rng(1).standard_normal(mesh.n1d(1, level) ** d)
    r[mesh.boundary_mask(d, 1, level)] = 0
    y = smoother.additive(d, 1, level, r)
    diag = mesh.operator_matrix(d, 1, level).diagonal()
    inner = mesh.interior_ids(d, 1, level)
    assert np.allclose(y[inner], r[inner] / diag, rtol=1e-14)


@pytest.mark.parametrize("d,k", [(2, 2), (2, 4), (3, 2)])
def test_additive_level1_is_exact_solve(d, k):
    r = np.random.default_rng(2).standard_normal(mesh.n1d(k, 1) ** d)
    r[mesh.boundary_mask(d, k, 1)] = 0
    y = smoother.additive(d, k, 1, r)
    A = mesh.operator_matrix(d, k, 1).toarray()
    inner = mesh.interior_ids(d, k, 1)
    assert np.allclose(A @ y[inner], r[inner], atol=1e-12)


def test_additive_symmetric_positive():
    d, k, level = 2, 2, 3
    rng = np.random.default_rng(3)
    N = mesh.n1d(k, level) ** d
    bm = mesh.boundary_mask(d, k, level)
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    u[bm] = v[bm] = 0
    Bu, Bv = smoother.additive(d, k, level, u), smoother.additive(d, k, level, v)
    assert abs(v @ Bu - u @ Bv) < 1e-12 * abs(u @ Bv)
    assert u @ Bu > 0 and v @ Bv > 0


@pytest.mark.parametrize("d,k,level", [(2, 2, 2), (2, 3, 2), (3, 1, 2)])
def test_colourised_equals_sequential_in_random_order(d, k, level):
    """Alg. 3 equals eq:simple-loop with patches taken in any order that keeps colours sequential."""
    rng = np.random.default_rng(4)
    N = mesh.n1d(k, level) ** d
    bm = mesh.boundary_mask(d, k, level)
    b, x = rng.standard_normal(N), rng.standard_normal(N)
    b[bm] = x[bm] = 0
    order = []
    for c in range(2 ** d):
        verts = list(mesh.patches_of_colour(d, level, c))
        rng.shuffle(verts)
        order += verts
    ref = smoother.sequential(d, k, level, b, x, order)
    got = smoother.multiplicative(d, k, level, b, x)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_boundary_identity_new_interior_independent_of_old():
    """Exact local solve: new x^I = A_j^{-1}(b^I - A^{IB} x^B) does not depend on old x^I (Sec. 4.1.3)."""
    d, k, level, c = 2, 3, 3, 0
    rng = np.random.default_rng(5)
    N = mesh.n1d(k, level) ** d
    bm = mesh.boundary_mask(d, k, level)
    b, x = rng.standard_normal(N), rng.standard_normal(N)
    b[bm] = x[bm] = 0
    x2 = x.copy()
    for v in mesh.patches_of_colour(d, level, c):
        I = mesh.patch_interior_ids(d, k, level, v)
        x2[I] = rng.standard_normal(len(I))
    y1 = smoother.colour_pass(d, k, level, b, x, c)
    y2 = smoother.colour_pass(d, k, level, b, x2, c)
    assert np.allclose(y1, y2, atol=1e-12)


def test_energy_error_decreases_each_colour():
    d, k, level = 2, 2, 3
    A = mesh.operator_matrix(d, k, level).toarray()
    inner = mesh.interior_ids(d, k, level)
    rng = np.random.default_rng(6)
    N = mesh.n1d(k, level) ** d
    b = np.zeros(N)
    b[inner] = rng.standard_normal(len(inner))
    xs = np.zeros(N)
    xs[inner] = np.linalg.solve(A, b[inner])
    x = np.zeros(N)
    err = lambda z: (z - xs)[inner] @ A @ (z - xs)[inner]
    e_prev = err(x)
    for c in range(4):
        x = smoother.colour_pass(d, k, level, b, x, c)
        e = err(x)
        assert e < e_prev
        e_prev = e


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2)])
def test_multiplicative_level1_is_exact(d, k):
    rng = np.random.default_rng(8)
    N = mesh.n1d(k, 1) ** d
    b = rng.standard_normal(N)
    b[mesh.boundary_mask(d, k, 1)] = 0
    x = smoother.multiplicative(d, k, 1, b, np.zeros(N))
    A = mesh.operator_matrix(d, k, 1).toarray()
    inner = mesh.interior_ids(d, k, 1)
    assert np.allclose(A @ x[inner], b[inner], atol=1e-12)


def test_local_patch_update_matches_colour_pass():
    d, k, level, c = 3, 2, 2, 5
    rng = np.random.default_rng(9)
    N = mesh.n1d(k, level) ** d
    bm = mesh.boundary_mask(d, k, level)
    b, x = rng.standard_normal(N), rng.standard_normal(N)
    b[bm] = x[bm] = 0
    y = smoother.colour_pass(d, k, level, b, x, c)
    for v in mesh.patches_of_colour(d, level, c):
        got = smoother.patch_update_local(d, k, level, x[mesh.patch_closure_ids(d, k, level, v)],
                                          b[mesh.patch_interior_ids(d, k, level, v)])
        assert np.allclose(got, y[mesh.patch_interior_ids(d, k, level, v)], atol=1e-12)


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 5), (3, 1), (3, 2), (3, 3)])
def test_a_ib_kronecker_blocks_equal_the_assembled_patch_matrix(d, k):
    """eq:A_ib_2d/3d: the Kronecker blocks reproduce the interior-row, boundary-column block of the
    closure matrix assembled from cell matrices, and their columns are exactly the boundary nodes."""
    h = 0.125
    A_ib, cols = smoother.a_ib_kronecker(d, k, h)
    Ac = smoother.patch_closure_matrix(d, k, h)
    I = smoother.patch_interior_local(d, k)
    B = np.setdiff1d(np.arange((2 * k + 1) ** d), I)
    assert np.array_equal(np.sort(cols), B)
    assert np.allclose(A_ib, Ac[np.ix_(I, cols)], atol=1e-13 * np.abs(Ac).max())


@pytest.mark.parametrize("d,k,level", [(2, 1, 3), (2, 3, 3), (3, 1, 3), (3, 2, 2), (3, 3, 2)])
def test_boundary_colour_pass_equals_the_fused_one(d, k, level):
    rng = np.random.default_rng(7)
    N = mesh.n1d(k, level) ** d
    bm = mesh.boundary_mask(d, k, level)
    b, x = rng.standard_normal(N), rng.standard_normal(N)
    b[bm] = x[bm] = 0
    for c in range(2 ** d):
        ref = smoother.colour_pass(d, k, level, b, x, c)
        got = smoother.colour_pass_boundary(d, k, level, b, x, c)
        assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max()), c
