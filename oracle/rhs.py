"""Right-hand sides of separable sine form and L2 errors (oracle, test infrastructure).

Paper passages: eq:matrix-def (b_i = int f phi_i) and Sec. 4.2 (manufactured
solution u = prod_i sin(pi x_i), error measured in L2).  A mode is
f(x) = c * prod_a sin(pi kappa_a x_a); for such f the load vector is the
Kronecker product of 1D load vectors.  All integrals use (k+1)-point Gauss per
cell direction unless a rule is named.
"""
import numpy as np

from . import basis, mesh


def load_vector_1d(k, level, kappa, nq=None):
    """g[i] = int_0^1 sin(pi kappa x) phi_i(x) dx over all nodes (cellwise Gauss)."""
    nq = k + 1 if nq is None else nq
    h = mesh.mesh_size(level)
    g_nodes = basis.gll_nodes(k)
    xq, wq = basis.gauss_rule(nq)
    V = basis.lagrange_values(g_nodes, xq)  # (k+1, nq)
    g = np.zeros(mesh.n1d(k, level))
    for c in range(2 ** level):
        xs = (c + xq) * h
        g[k * c:k * c + k + 1] += V @ (wq * h * np.sin(np.pi * kappa * xs))
    return g


def rhs_sine_modes(d, k, level, kappas, coefs):
    """b = sum_m coefs[m] * (x)_a g_{kappas[m][a]}; full-grid vector with zero boundary."""
    n = mesh.n1d(k, level)
    B = np.zeros((n,) * d)
    for kap, c in zip(kappas, coefs):
        T = np.array(c, dtype=np.float64).reshape((1,) * d)
        for a in range(d):
            shape = [1] * d
            shape[d - 1 - a] = n
            T = T * load_vector_1d(k, level, kap[a]).reshape(shape)
        B = B + T
    b = B.reshape(-1)
    b[mesh.boundary_mask(d, k, level)] = 0.0
    return b


def rhs_constant(d, k, level):
    """b for f = 1 (the right-hand side of the FMG tests, Sec. 4.1): Kronecker product of the
    1D load vector of 1, whose entries are the row sums of h * Mhat over the cells."""
    _, Mhat = basis.reference_matrices(k)
    h = mesh.mesh_size(level)
    g = np.zeros(mesh.n1d(k, level))
    for c in range(2 ** level):
        g[k * c:k * c + k + 1] += h * Mhat.sum(1)
    B = np.ones((1,) * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = len(g)
        B = B * g.reshape(shape)
    b = B.reshape(-1)
    b[mesh.boundary_mask(d, k, level)] = 0
    return b


def rhs_bruteforce(d, k, level, f):
    """b_i = int f phi_i by d-dim cellwise Gauss quadrature, point by point (tiny meshes; pins)."""
    import itertools
    h = mesh.mesh_size(level)
    g_nodes = basis.gll_nodes(k)
    xq, wq = basis.gauss_rule(k + 1)
    V = basis.lagrange_values(g_nodes, xq)
    b = np.zeros(mesh.n1d(k, level) ** d)
    for cell in itertools.product(range(2 ** level), repeat=d):
        cell = cell[::-1]  # (c_0, ..., c_{d-1})
        ids = mesh.cell_dof_ids(d, k, level, cell)
        loc = np.zeros((k + 1,) * d)
        for q in itertools.product(range(k + 1), repeat=d):  # (q_{d-1},...,q_0)
            pt = [(cell[a] + xq[q[d - 1 - a]]) * h for a in range(d)]
            w = np.prod([wq[qq] for qq in q]) * h ** d
            fv = f(pt)
            for li in itertools.product(range(k + 1), repeat=d):
                phi = np.prod([V[li[d - 1 - a], q[d - 1 - a]] for a in range(d)])
                loc[li] += w * fv * phi
        b[ids] += loc.reshape(-1)
    b[mesh.boundary_mask(d, k, level)] = 0.0
    return b


def exact_solution_coefs(kappas, coefs):
    """Coefficients of u for -Lap u = f with f = sum c_m prod sin(pi kappa x): c_m / (pi^2 |kappa|^2)."""
    return [c / (np.pi ** 2 * float(np.dot(kap, kap))) for kap, c in zip(kappas, coefs)]


def l2_error(d, k, level, x, kappas, ucoefs, nq=None):
    """|| u - u_h ||_{L2} with u = sum ucoefs[m] prod_a sin(pi kappa_ma x_a), cellwise Gauss."""
    nq = k + 1 if nq is None else nq
    n = mesh.n1d(k, level)
    h = mesh.mesh_size(level)
    g_nodes = basis.gll_nodes(k)
    xq, wq = basis.gauss_rule(nq)
    V = basis.lagrange_values(g_nodes, xq)  # (k+1, nq)
    # interpolation of nodal values to quadrature points, axis by axis:
    # global 1D matrix E (n_cells*nq x n) with E[c*nq+q, k*c+i] = V[i, q]
    nc = 2 ** level
    E = np.zeros((nc * nq, n))
    for c in range(nc):
        E[c * nq:(c + 1) * nq, k * c:k * c + k + 1] = V.T
    X = np.asarray(x).reshape((n,) * d)
    for a in range(d):
        X = mesh.apply_1d(E, X, a, d)
    xs = ((np.arange(nc)[:, None] + xq[None, :]) * h).reshape(-1)
    ws = np.tile(wq * h, nc)
    U = np.zeros((nc * nq,) * d)
    for kap, c in zip(kappas, ucoefs):
        T = np.array(c).reshape((1,) * d)
        for a in range(d):
            shape = [1] * d
            shape[d - 1 - a] = nc * nq
            T = T * np.sin(np.pi * kap[a] * xs).reshape(shape)
        U = U + T
    W = np.ones((1,) * d)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = nc * nq
        W = W * ws.reshape(shape)
    return float(np.sqrt(np.sum(W * (U - X) ** 2)))


def rhs_sine_modes_at(d, k, level, kappas, coefs, coords):
    """Entries of rhs_sine_modes at the nodes `coords` ((S, d) array of (c_0, ..., c_{d-1})) only,
    from the same 1D load vectors; 0 on Dirichlet nodes.  For meshes too large to hold b."""
    n = mesh.n1d(k, level)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d)
    cache = {}
    out = np.zeros(len(coords))
    for kap, c in zip(kappas, coefs):
        t = np.full(len(coords), float(c))
        for a in range(d):
            key = int(kap[a])
            if key not in cache:
                cache[key] = load_vector_1d(k, level, key)
            t = t * cache[key][coords[:, a]]
        out += t
    out[np.any((coords == 0) | (coords == n - 1), axis=1)] = 0.0
    return out
