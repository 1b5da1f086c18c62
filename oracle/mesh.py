"""Uniform level meshes, lexicographic DoF layout, global operator, vertex patches (oracle).

Paper passages: Sec. 2 (mesh hierarchy by uniform refinement, eq:linear_system,
eq:matrix-def, Dirichlet DoFs eliminated), Sec. 2.4 eq:tensorproduct_2d/3d
(Kronecker structure), Sec. 2.2 (vertex patches, Fig. 2 colouring), Sec. 3.1.2
(global lexicographic numbering, Fig. 4).
"""
import functools
import itertools

import numpy as np
import scipy.sparse as sp

from . import basis


def n1d(k, level):
    """Nodes per direction on level `level` (2**level cells, k*2**level + 1 nodes)."""
    return k * 2 ** level + 1


def mesh_size(level):
    return 2.0 ** (-level)


@functools.lru_cache(maxsize=None)
def global_1d_matrices(k, level):
    """Assembled 1D stiffness A1 = sum_cells Ahat/h and mass M1 = sum_cells h*Mhat (all nodes)."""
    Ahat, Mhat = basis.reference_matrices(k)
    h = mesh_size(level)
    n = n1d(k, level)
    A1 = np.zeros((n, n))
    M1 = np.zeros((n, n))
    for c in range(2 ** level):
        s = slice(k * c, k * c + k + 1)
        A1[s, s] += Ahat / h
        M1[s, s] += h * Mhat
    return sp.csr_matrix(A1), sp.csr_matrix(M1)


@functools.lru_cache(maxsize=None)
def boundary_mask(d, k, level):
    """Boolean full-grid mask of Dirichlet boundary nodes (flat, x0 fastest)."""
    n = n1d(k, level)
    on_b = np.zeros(n, dtype=bool)
    on_b[0] = on_b[-1] = True
    mask = np.zeros((n,) * d, dtype=bool)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n
        mask |= on_b.reshape(shape)
    return mask.reshape(-1)


def interior_ids(d, k, level):
    return np.flatnonzero(~boundary_mask(d, k, level))


def apply_1d(mat, X, axis, d):
    """Apply the 1D matrix `mat` along coordinate axis `axis` of the d-dim array X."""
    ax = d - 1 - axis
    Xm = np.moveaxis(X, ax, 0)
    shp = Xm.shape
    Y = mat @ Xm.reshape(shp[0], -1)
    return np.moveaxis(np.asarray(Y).reshape((mat.shape[0],) + shp[1:]), 0, ax)


def apply_operator(d, k, level, x):
    """y = A_level x for the Poisson stiffness matrix (eq:matrix-def), full-grid vectors.

    A = sum_dir (x)_a (A1 if a == dir else M1) (eq:tensorproduct on the whole
    mesh).  Boundary entries of x are ignored; boundary entries of y are 0.
    """
    n = n1d(k, level)
    A1, M1 = global_1d_matrices(k, level)
    bmask = boundary_mask(d, k, level)
    X = np.where(bmask, 0.0, np.asarray(x, dtype=np.float64)).reshape((n,) * d)
    Y = np.zeros_like(X)
    for direction in range(d):
        T = X
        for a in range(d):
            T = apply_1d(A1 if a == direction else M1, T, a, d)
        Y += T
    y = Y.reshape(-1)
    y[bmask] = 0.0
    return y


def operator_matrix(d, k, level):
    """Explicit sparse interior matrix A (rows/cols = interior nodes in lexicographic order)."""
    A1, M1 = global_1d_matrices(k, level)
    inner = slice(1, n1d(k, level) - 1)
    A1 = A1[inner, inner]
    M1 = M1[inner, inner]
    total = None
    for direction in range(d):
        term = None
        for a in reversed(range(d)):  # leftmost factor = slowest axis x_{d-1}
            f = A1 if a == direction else M1
            term = f if term is None else sp.kron(term, f)
        total = term if total is None else total + term
    return sp.csr_matrix(total)


def assembled_matrix_bruteforce(d, k, level):
    """Global matrix by summing cell matrices (sum_K R_K^T A^K R_K), all nodes, dense.

    Used to pin the Kronecker form on tiny meshes.
    """
    n = n1d(k, level)
    h = mesh_size(level)
    AK = basis.cell_matrix(d, k, h)
    N = n ** d
    A = np.zeros((N, N))
    for cell in itertools.product(range(2 ** level), repeat=d):  # (c_{d-1},...,c_0)
        ids = cell_dof_ids(d, k, level, cell[::-1])
        A[np.ix_(ids, ids)] += AK
    return A


def flat_index(d, k, level, coords):
    """Flat full-grid index of node coords (c_0, ..., c_{d-1}), x0 fastest."""
    n = n1d(k, level)
    idx = 0
    for a in reversed(range(d)):
        idx = idx * n + int(coords[a])
    return idx


def box_ids(d, k, level, lo, length):
    """Flat indices of the node box [lo_a, lo_a + length) per axis, lexicographic, x0 fastest."""
    n = n1d(k, level)
    ranges = [np.arange(lo[a], lo[a] + length) for a in range(d)]
    ids = np.zeros([length] * d, dtype=np.int64)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = length
        ids = ids + ranges[a].reshape(shape) * n ** a
    return ids.reshape(-1)


def cell_dof_ids(d, k, level, cell):
    """DoFs of cell `cell` = (c_0, ..., c_{d-1}): (k+1)^d nodes."""
    return box_ids(d, k, level, [k * c for c in cell], k + 1)


# ---------------------------------------------------------------- vertex patches

def patch_vertices(d, level):
    """All interior vertices v in {1..2**level-1}^d as rows (v_0, ..., v_{d-1})."""
    m = 2 ** level
    return np.array([t[::-1] for t in itertools.product(range(1, m), repeat=d)], dtype=np.int64)


def patch_colour(v):
    """Colour of the vertex patch at v (Fig. 2: colours shift by one cell per direction)."""
    return int(sum(((int(vi) - 1) % 2) << a for a, vi in enumerate(v)))


def patches_of_colour(d, level, colour):
    verts = patch_vertices(d, level)
    keep = [i for i, v in enumerate(verts) if patch_colour(v) == colour]
    return verts[keep]


def patch_closure_ids(d, k, level, v):
    """Closure DoFs of the patch of vertex v: (2k+1)^d nodes [k(v_a-1), k(v_a+1)] (Fig. 1 left)."""
    return box_ids(d, k, level, [k * (int(va) - 1) for va in v], 2 * k + 1)


def patch_interior_ids(d, k, level, v):
    """Interior DoFs of the patch: (2k-1)^d nodes strictly inside the patch (Fig. 1 right)."""
    return box_ids(d, k, level, [k * (int(va) - 1) + 1 for va in v], 2 * k - 1)


def patch_box_ids_many(d, k, level, verts, interior):
    """Closure (interior=False) or interior (True) DoFs of many patches, one patch per row.

    Row p lists the same nodes in the same order as patch_closure_ids / patch_interior_ids of
    verts[p]."""
    verts = np.asarray(verts, dtype=np.int64).reshape(-1, d)
    n = n1d(k, level)
    first = 1 if interior else 0
    length = 2 * k - 1 if interior else 2 * k + 1
    base = np.zeros(len(verts), dtype=np.int64)
    for a in range(d):
        base += (k * (verts[:, a] - 1) + first) * n ** a
    return base[:, None] + box_ids(d, k, level, [0] * d, length)[None, :]


def operator_rows(d, k, level, coords, x, absolute=False):
    """(A x)_i for the nodes i at `coords` ((S, d) array of (c_0, ..., c_{d-1})), one row at a time.

    absolute=True returns instead sum_dir ((x)_a |A1 or M1|) |x| on those rows: the sum of the
    magnitudes of all products that make up (A x)_i in the Kronecker-sum form.  A computed row
    sum differs from the exact one by at most gamma_n times this (the standard bound for
    floating-point sums of products, with n the depth of the summation), which is what
    tolerances on computed rows are measured against.

    `x` is any object indexable by flat node ids (a full-grid vector, or a device tensor).  A row
    of A = sum_dir (x)_a (A1 or M1) couples node i only to the nodes whose coordinate differs by at
    most k on every axis, so each row takes the (2k+1)^d box around i; Dirichlet nodes of x count
    as 0 and Dirichlet rows are 0 (as in apply_operator).
    """
    n = n1d(k, level)
    A1, M1 = global_1d_matrices(k, level)
    A1, M1 = A1.toarray() if n <= 4097 else A1, M1.toarray() if n <= 4097 else M1
    if absolute:
        A1, M1 = abs(A1), abs(M1)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d)
    out = np.zeros(len(coords))
    for s, c in enumerate(coords):
        if np.any(c == 0) or np.any(c == n - 1):
            continue
        lo = [max(int(c[a]) - k, 1) for a in range(d)]
        hi = [min(int(c[a]) + k, n - 2) for a in range(d)]
        ranges = [np.arange(lo[a], hi[a] + 1) for a in range(d)]
        ids = np.zeros([len(r) for r in reversed(ranges)], dtype=np.int64)
        for a in range(d):
            shape = [1] * d
            shape[d - 1 - a] = len(ranges[a])
            ids = ids + ranges[a].reshape(shape) * n ** a
        X = np.asarray(x[ids.reshape(-1)], dtype=np.float64).reshape(ids.shape)
        if absolute:
            X = np.abs(X)
        total = 0.0
        for direction in range(d):
            T = X
            for a in range(d):
                row = (A1 if a == direction else M1)[int(c[a]), ranges[a]]
                row = np.asarray(row.todense() if hasattr(row, "todense") else row).reshape(1, -1)
                T = apply_1d(row, T, a, d)
            total += float(np.asarray(T).reshape(-1)[0])
        out[s] = total
    return out
