"""Exact discrete solution x = A_L^{-1} b by a direct method (oracle, test infrastructure).

Paper passages: Sec. 2, eq:linear_system (the discrete Poisson system A u = b
with Dirichlet DoFs eliminated) and eq:tensorproduct_2d/3d (on a uniform
Cartesian mesh A is a Kronecker sum of the global 1D stiffness A1 and mass M1
matrices).  For a Kronecker sum the generalized eigenvectors of the 1D pencil,
A1 S = M1 S Lambda with S^T M1 S = I, diagonalise the whole operator:

    A^{-1} = (S x .. x S) (Lambda (+) .. (+) Lambda)^{-1} (S x .. x S)^T,

the same identity the paper uses on one patch (eq:inverse2d/3d), here applied
to the interior DoFs of the whole mesh.  It is a direct solve, not the
method's iteration, and serves as the reference solution of the solver tests.
The eigen-decomposition is LAPACK's (scipy.linalg.eigh); the tests pin the
result against a sparse LU solve of the assembled matrix on small meshes.
"""
import functools

import numpy as np
import scipy.linalg as sla

from . import mesh


@functools.lru_cache(maxsize=8)
def _pencil(k, level):
    A1, M1 = mesh.global_1d_matrices(k, level)
    inner = slice(1, mesh.n1d(k, level) - 1)
    lam, S = sla.eigh(A1[inner, inner].toarray(), M1[inner, inner].toarray())
    return lam, S


def exact_solve(d, k, level, b):
    """x = A_level^{-1} b on the interior DoFs; full-grid vectors, boundary entries of x are 0.

    Boundary entries of b are ignored (Dirichlet elimination)."""
    lam, S = _pencil(k, level)
    n = mesh.n1d(k, level)
    m = n - 2
    B = np.asarray(b, dtype=np.float64).reshape((n,) * d)[(slice(1, n - 1),) * d]
    T = B
    for a in range(d):
        T = mesh.apply_1d(S.T, T, a, d)
    den = np.zeros((m,) * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = m
        den = den + lam.reshape(shape)
    T = T / den
    for a in range(d):
        T = mesh.apply_1d(S, T, a, d)
    X = np.zeros((n,) * d)
    X[(slice(1, n - 1),) * d] = T
    return X.reshape(-1)
