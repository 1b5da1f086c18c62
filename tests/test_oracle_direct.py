"""Pins of the oracle's exact discrete solve and of its batched patch updates.

The exact solve (global Kronecker eigen-decomposition) is checked against a
sparse LU solve of the assembled interior matrix and against A^{-1}(A x) = x;
the batched local patch update (localised residual, Sec. 2.2) is checked against
the colour pass that forms one global residual per colour.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import direct, mesh, smoother


@pytest.mark.parametrize("d,k,L", [(2, 1, 3), (2, 2, 3), (2, 4, 2), (2, 7, 2), (3, 1, 3), (3, 2, 2), (3, 3, 2),
                                   (3, 5, 1)])
def test_exact_solve_equals_sparse_lu(d, k, L):
    b = synth.random_interior(d, k, L, 5)
    inner = mesh.interior_ids(d, k, L)
    ref = spla.spsolve(mesh.operator_matrix(d, k, L).tocsc(), b[inner])
    x = direct.exact_solve(d, k, L, b)
    assert np.linalg.norm(x[inner] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(x[mesh.boundary_mask(d, k, L)] == 0.0)


@pytest.mark.parametrize("d,k,L", [(2, 3, 6), (3, 2, 4), (3, 4, 3)])
def test_exact_solve_inverts_the_operator(d, k, L):
    """A^{-1}(A x) = x and b - A(A^{-1} b) = 0 through the axis-wise operator, boundary of b ignored."""
    x = synth.random_interior(d, k, L, 6)
    y = direct.exact_solve(d, k, L, mesh.apply_operator(d, k, L, x))
    assert np.linalg.norm(y - x) <= 1e-11 * np.linalg.norm(x)
    b = synth.random_interior(d, k, L, 7)
    bg = b.copy()
    bg[mesh.boundary_mask(d, k, L)] = 4.0
    r = b - mesh.apply_operator(d, k, L, direct.exact_solve(d, k, L, bg))
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)


def test_exact_solve_reproduces_a_discrete_polynomial():
    """The bubble u = prod x_a(1 - x_a) lies in Q_2: its nodal vector solves A u = A u exactly."""
    d, k, L = 3, 2, 3
    t = np.linspace(0.0, 1.0, mesh.n1d(k, L))  # Q2 GLL nodes on a uniform mesh are equispaced
    g = t * (1 - t)
    u = (g[:, None, None] * g[None, :, None] * g[None, None, :]).reshape(-1)
    assert np.allclose(direct.exact_solve(d, k, L, mesh.apply_operator(d, k, L, u)), u, atol=1e-13)


@pytest.mark.parametrize("d,k,L", [(2, 3, 3), (3, 2, 2), (3, 4, 2)])
def test_batched_local_updates_equal_the_colour_pass(d, k, L):
    b = synth.random_interior(d, k, L, 8)
    x = synth.random_interior(d, k, L, 9)
    for c in range(2 ** d):
        verts = mesh.patches_of_colour(d, L, c)
        if len(verts) == 0:
            continue
        C = mesh.patch_box_ids_many(d, k, L, verts, interior=False)
        I = mesh.patch_box_ids_many(d, k, L, verts, interior=True)
        for p, v in enumerate(verts):
            assert np.array_equal(C[p], mesh.patch_closure_ids(d, k, L, v))
            assert np.array_equal(I[p], mesh.patch_interior_ids(d, k, L, v))
        got = smoother.patch_update_local_many(d, k, L, x[C], b[I])
        ref = smoother.colour_pass(d, k, L, b, x, c)[I]
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        # the additive local solve against the patch block cut out of the global interior matrix
        add = smoother.patch_solve_many(d, k, L, b[I])
        for p in (0, len(verts) - 1):
            ref = np.linalg.solve(smoother.patch_matrix_from_global(d, k, L, verts[p]), b[I[p]])
            assert np.max(np.abs(add[p] - ref)) <= 1e-12 * np.max(np.abs(ref))
