"""Vertex-patch Schwarz smoothers with dense-LU local solves (oracle, test infrastructure).

Paper passages: Sec. 2.2 -- eq:residual and eq:local-solver (subspace correction
s_j), eq:simple-loop (sequential multiplicative smoother), the localised residual
r_j = R_j b - Abar_j Rbar_j x, and Alg. 3 (colourised smoother: sequential over
colours, parallel inside a colour).  The local matrix A_j is the restriction of
eq:matrix-def to the patch interior; here it is formed explicitly and solved by
dense LU (the plain definition the fast-diagonalisation method reaches).
"""
import functools

import numpy as np
import scipy.linalg as sla

from . import basis, mesh


def patch_closure_matrix(d, k, h):
    """Closure matrix of a vertex patch: sum over its 2^d cells of R_K^T A^K R_K.

    Rows/cols are the (2k+1)^d closure nodes, lexicographic with x0 fastest.  Its
    interior rows equal the rows of the global matrix (interior basis functions
    are supported inside the patch), which the tests check.
    """
    n = 2 * k + 1
    AK = basis.cell_matrix(d, k, h)
    A = np.zeros((n ** d, n ** d))
    for cell in np.ndindex(*([2] * d)):  # (c_{d-1},...,c_0) in {0,1}^d
        lo = [k * c for c in cell[::-1]]
        ranges = [np.arange(lo[a], lo[a] + k + 1) for a in range(d)]
        ids = np.zeros([k + 1] * d, dtype=np.int64)
        for a in range(d):
            shape = [1] * d
            shape[d - 1 - a] = k + 1
            ids = ids + ranges[a].reshape(shape) * n ** a
        ids = ids.reshape(-1)
        A[np.ix_(ids, ids)] += AK
    return A


def patch_interior_local(d, k):
    """Local indices (within the closure numbering) of the (2k-1)^d patch-interior nodes."""
    n = 2 * k + 1
    inner = np.arange(1, n - 1)
    ids = np.zeros([n - 2] * d, dtype=np.int64)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n - 2
        ids = ids + inner.reshape(shape) * n ** a
    return ids.reshape(-1)


@functools.lru_cache(maxsize=None)
def patch_matrices(d, k, level):
    """(Abar_j, A_j): interior rows x closure cols, and interior x interior (same for every patch)."""
    Ac = patch_closure_matrix(d, k, mesh.mesh_size(level))
    I = patch_interior_local(d, k)
    return Ac[I, :], Ac[np.ix_(I, I)]


def patch_matrix_from_global(d, k, level, v):
    """A_j = A[I_j, I_j] cut out of the explicit global interior matrix (tiny meshes only)."""
    A = mesh.operator_matrix(d, k, level)
    pos = np.full(mesh.n1d(k, level) ** d, -1, dtype=np.int64)
    inner = mesh.interior_ids(d, k, level)
    pos[inner] = np.arange(len(inner))
    J = pos[mesh.patch_interior_ids(d, k, level, v)]
    return A[J][:, J].toarray()


@functools.lru_cache(maxsize=None)
def _patch_lu(d, k, level):
    """Dense LU factors of A_j (identical for every patch of the level)."""
    return sla.lu_factor(patch_matrices(d, k, level)[1])


@functools.lru_cache(maxsize=None)
def _colour_index_arrays(d, k, level, colour):
    verts = mesh.patches_of_colour(d, level, colour)
    if len(verts) == 0:
        return np.zeros((0, (2 * k - 1) ** d), dtype=np.int64)
    return np.stack([mesh.patch_interior_ids(d, k, level, v) for v in verts])


def additive(d, k, level, r):
    """y = sum_j R_j^T A_j^{-1} R_j r (one undamped additive Schwarz application).

    Every A_j is the same matrix on a uniform mesh; it is factored once and all
    patches are solved with it.
    """
    lu = _patch_lu(d, k, level)
    r = np.asarray(r, dtype=np.float64)
    y = np.zeros_like(r)
    for colour in range(2 ** d):
        I = _colour_index_arrays(d, k, level, colour)
        if len(I) == 0:
            continue
        sol = sla.lu_solve(lu, r[I].T)  # one column per patch
        np.add.at(y, I.T, sol)
    return y


def colour_pass(d, k, level, b, x, colour, lu=None):
    """One colour of Alg. 3: for all patches j of the colour, x += R_j^T A_j^{-1} (R_j (b - A x)).

    Same-colour patches are disjoint, so one global residual serves them all.
    """
    if lu is None:
        lu = _patch_lu(d, k, level)
    I = _colour_index_arrays(d, k, level, colour)
    if len(I) == 0:
        return x
    r = np.asarray(b) - mesh.apply_operator(d, k, level, x)
    x = x.copy()
    x[I] += sla.lu_solve(lu, r[I].T).T
    return x


def patch_1d_matrices(k, h):
    """1D patch matrices on the 2k+1 nodes of two cells of size h: stiffness (Ahat/h) and
    mass (h*Mhat) assembled over both cells."""
    Ahat, Mhat = basis.reference_matrices(k)
    n = 2 * k + 1
    A, M = np.zeros((n, n)), np.zeros((n, n))
    for c in (0, 1):
        s = slice(k * c, k * c + k + 1)
        A[s, s] += Ahat / h
        M[s, s] += h * Mhat
    return A, M


def a_ib_kronecker(d, k, h):
    """A^{IB} of a vertex patch from the Kronecker blocks of eq:A_ib_2d / eq:A_ib_3d.

    The boundary closure nodes fall into d groups: group g holds the nodes whose axis-g index
    is on the patch boundary, whose higher axes are interior and whose lower axes are
    arbitrary.  On group g every direction term of the operator is a Kronecker product of
    1D blocks: interior rows throughout, boundary columns on axis g, all columns below g and
    interior columns above g.  Returns (A^{IB}, closure-local ids of its columns).
    """
    A1, M1 = patch_1d_matrices(k, h)
    n = 2 * k + 1
    inner, bnd, every = np.arange(1, n - 1), np.array([0, n - 1]), np.arange(n)
    blocks, cols = [], []
    for g in range(d):
        colsets = [every if a < g else (bnd if a == g else inner) for a in range(d)]
        total = 0.0
        for direction in range(d):
            mats = [(A1 if a == direction else M1)[np.ix_(inner, colsets[a])] for a in range(d)]
            total = total + basis._kron_axes(mats)
        blocks.append(total)
        ids = np.zeros([len(colsets[a]) for a in reversed(range(d))], dtype=np.int64)
        for a in range(d):
            shape = [1] * d
            shape[d - 1 - a] = len(colsets[a])
            ids = ids + colsets[a].reshape(shape) * n ** a
        cols.append(ids.reshape(-1))
    return np.hstack(blocks), np.concatenate(cols)


def colour_pass_boundary(d, k, level, b, x, colour):
    """One colour of Alg. 3 in the form of Sec. 4.1.3: x_j^I <- A_j^{-1}(b_j^I - A^{IB} x_j^B).

    Reads only the boundary nodes of each patch closure (Dirichlet nodes count as 0)."""
    verts = mesh.patches_of_colour(d, level, colour)
    x = np.asarray(x, dtype=np.float64).copy()
    if len(verts) == 0:
        return x
    A_ib, bcols = a_ib_kronecker(d, k, mesh.mesh_size(level))
    xz = x.copy()
    xz[mesh.boundary_mask(d, k, level)] = 0.0
    C = np.stack([mesh.patch_closure_ids(d, k, level, v) for v in verts])
    I = np.stack([mesh.patch_interior_ids(d, k, level, v) for v in verts])
    rhs = np.asarray(b)[I] - xz[C[:, bcols]] @ A_ib.T
    x[I] = sla.lu_solve(_patch_lu(d, k, level), rhs.T).T
    return x


def multiplicative(d, k, level, b, x, reverse=False):
    """Colourised multiplicative vertex-patch smoother S_l(x, b) (Alg. 3).

    Colours run 0..2^d-1, or in reverse order when `reverse` (post-smoothing).
    """
    lu = _patch_lu(d, k, level)
    x = np.asarray(x, dtype=np.float64).copy()
    x[mesh.boundary_mask(d, k, level)] = 0.0
    order = range(2 ** d - 1, -1, -1) if reverse else range(2 ** d)
    for colour in order:
        x = colour_pass(d, k, level, b, x, colour, lu)
    return x


def sequential(d, k, level, b, x, order):
    """eq:simple-loop: x <- s_{j_J} o ... o s_{j_1}(x), one patch at a time, global residual each step."""
    _, Aj = patch_matrices(d, k, level)
    x = np.asarray(x, dtype=np.float64).copy()
    for v in order:
        r = np.asarray(b) - mesh.apply_operator(d, k, level, x)
        I = mesh.patch_interior_ids(d, k, level, v)
        x[I] += np.linalg.solve(Aj, r[I])
    return x


def patch_update_local(d, k, level, x_closure, b_interior):
    """New interior values of one patch from its local data only (localised residual, Sec. 2.2).

    x_closure: (2k+1)^d values of x on the patch closure (Dirichlet nodes must be 0);
    b_interior: (2k-1)^d values of b on the patch interior.
    Returns x^I + A_j^{-1}(b^I - Abar_j x_closure).
    """
    Abar, Aj = patch_matrices(d, k, level)
    I = patch_interior_local(d, k)
    r = np.asarray(b_interior) - Abar @ np.asarray(x_closure)
    return np.asarray(x_closure)[I] + np.linalg.solve(Aj, r)


def patch_update_local_many(d, k, level, x_closures, b_interiors):
    """patch_update_local for many patches at once, one patch per row.

    x_closures: (P, (2k+1)^d) closure values (Dirichlet nodes 0); b_interiors: (P, (2k-1)^d).
    Returns the (P, (2k-1)^d) new interior values x^I + A_j^{-1}(b^I - Abar_j x_closure).
    """
    Abar, _ = patch_matrices(d, k, level)
    I = patch_interior_local(d, k)
    X = np.asarray(x_closures, dtype=np.float64)
    r = np.asarray(b_interiors, dtype=np.float64) - X @ Abar.T
    return X[:, I] + sla.lu_solve(_patch_lu(d, k, level), r.T).T


def patch_solve_many(d, k, level, r_interiors):
    """A_j^{-1} r for many patch-interior vectors r (one per row): the local solve of the additive
    smoother (eq:local-solver), by the dense LU of the explicit patch matrix."""
    return sla.lu_solve(_patch_lu(d, k, level), np.asarray(r_interiors, dtype=np.float64).T).T
