"""Fast-diagonalisation inverse of the patch matrix (oracle cross-check only).

Paper passage: Sec. 2.4, eq:tensorproduct_2d/3d, eq:inverse2d/3d and
eq:fast_inverse.  The 1D patch stiffness/mass pair (on the 2k-1 interior nodes of
two cells) is diagonalised by the generalised eigenproblem A S = M S Lambda with
S^T M S = I; the d-dim inverse is (S x..x S)(sum of Lambdas)^{-1}(S x..x S)^T.
The oracle itself solves patches by dense LU; this module exists to show, in the
tests, that the formula the GPU kernels implement equals that dense inverse.
"""
import numpy as np
import scipy.linalg as sla

from . import smoother


def patch_1d_matrices(k, h):
    """1D patch stiffness and mass restricted to the 2k-1 patch-interior nodes."""
    Ac = smoother.patch_closure_matrix(1, k, h)  # d = 1: closure of two 1D cells
    Mc = _patch_closure_mass_1d(k, h)
    inner = slice(1, 2 * k)
    return Ac[inner, inner], Mc[inner, inner]


def _patch_closure_mass_1d(k, h):
    from . import basis
    _, Mhat = basis.reference_matrices(k)
    n = 2 * k + 1
    M = np.zeros((n, n))
    for c in range(2):
        s = slice(k * c, k * c + k + 1)
        M[s, s] += h * Mhat
    return M


def eigen_1d(k, h):
    """(S, lam) with A S = M S diag(lam) and S^T M S = I (eq:fast_inverse)."""
    A, M = patch_1d_matrices(k, h)
    lam, S = sla.eigh(A, M)
    return S, lam


def inverse(d, k, h):
    """Dense matrix (S x..x S) diag(1 / sum lam) (S x..x S)^T (eq:inverse2d/3d)."""
    S, lam = eigen_1d(k, h)
    m = len(lam)
    Sd = np.ones((1, 1))
    for _ in range(d):
        Sd = np.kron(Sd, S)
    lsum = np.zeros([m] * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = m
        lsum = lsum + lam.reshape(shape)
    return Sd @ np.diag(1.0 / lsum.reshape(-1)) @ Sd.T
