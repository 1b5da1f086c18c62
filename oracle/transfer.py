"""Grid transfer between levels (oracle, test infrastructure).

Paper passage: Sec. 2.1 -- prolongation is the embedding V_{l-1} -> V_l realised
by polynomial interpolation of the coarse function at the fine support points;
restriction is its transpose.  Both act on the interior (Dirichlet) DoFs only.
"""
import functools

import numpy as np

from . import basis, mesh


@functools.lru_cache(maxsize=None)
def prolongation_1d(k, level_fine):
    """P1[i, J] = phi^coarse_J(x^fine_i): coarse global Lagrange basis at fine nodes (all nodes)."""
    lc = level_fine - 1
    hc = mesh.mesh_size(lc)
    nf, nc = mesh.n1d(k, level_fine), mesh.n1d(k, lc)
    g = basis.gll_nodes(k)
    # physical fine node coordinates
    hf = mesh.mesh_size(level_fine)
    xf = np.concatenate([c * hf + g[:-1] * hf for c in range(2 ** level_fine)] + [[1.0]])
    P = np.zeros((nf, nc))
    for i, x in enumerate(xf):
        cell = min(int(np.floor(x / hc + 1e-12)), 2 ** lc - 1)
        xi = x / hc - cell  # position in the coarse reference cell
        vals = basis.lagrange_values(g, [xi])[:, 0]
        for a in range(k + 1):
            P[i, k * cell + a] = vals[a]
    P[np.abs(P) < 1e-15] = 0.0
    return P


def prolongate(d, k, level_fine, e):
    """Fine full-grid vector P e (P = P1 x..x P1), boundary entries 0."""
    P1 = prolongation_1d(k, level_fine)
    nc = mesh.n1d(k, level_fine - 1)
    E = np.where(mesh.boundary_mask(d, k, level_fine - 1), 0.0, e).reshape((nc,) * d)
    for a in range(d):
        E = mesh.apply_1d(P1, E, a, d)
    out = E.reshape(-1)
    out[mesh.boundary_mask(d, k, level_fine)] = 0.0
    return out


def restrict(d, k, level_fine, r):
    """Coarse full-grid vector P^T r, boundary entries 0."""
    P1 = prolongation_1d(k, level_fine)
    nf = mesh.n1d(k, level_fine)
    R = np.where(mesh.boundary_mask(d, k, level_fine), 0.0, r).reshape((nf,) * d)
    for a in range(d):
        R = mesh.apply_1d(P1.T, R, a, d)
    out = R.reshape(-1)
    out[mesh.boundary_mask(d, k, level_fine - 1)] = 0.0
    return out
