"""1D support points, quadrature and Q_k reference matrices (oracle, test infrastructure).

Paper passages: Sec. 2 (Q_k Lagrange elements on Gauss-Lobatto support points,
eq:weak_form, eq:matrix-def) and Sec. 2.3 (eq:mf0 / eq:mf: on a Cartesian cell
the cell stiffness matrix is a Kronecker sum of 1D stiffness and mass matrices).
"""
import functools
import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k):
    """k+1 Gauss-Lobatto support points on [0, 1] (Sec. 2: support points of Q_k).

    Interior points are the roots of P_k' on [-1, 1], mapped by t -> (t+1)/2.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    inner = npleg.Legendre.basis(k).deriv().roots() if k > 1 else np.array([])
    t = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    return (t + 1.0) / 2.0


def gauss_rule(nq):
    """nq-point Gauss-Legendre rule on [0, 1] (exact for degree 2*nq-1)."""
    t, w = npleg.leggauss(nq)
    return (t + 1.0) / 2.0, w / 2.0


def lagrange_values(nodes, x):
    """V[i, q] = phi_i(x_q) for the Lagrange polynomials of `nodes` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((n, len(x)))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[i, q] = phi_i'(x_q): derivative of the product formula, term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((n, len(x)))
    for i in range(n):
        for l in range(n):
            if l == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[l]))
            for j in range(n):
                if j != i and j != l:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return D


@functools.lru_cache(maxsize=None)
def reference_matrices(k):
    """1D reference stiffness Ahat_ij = int_0^1 phi_i' phi_j' and mass Mhat_ij = int_0^1 phi_i phi_j.

    (k+1)-point Gauss quadrature integrates both exactly (integrands of degree <= 2k).
    """
    g = gll_nodes(k)
    xq, wq = gauss_rule(k + 1)
    V = lagrange_values(g, xq)
    D = lagrange_derivatives(g, xq)
    Ahat = (D * wq) @ D.T
    Mhat = (V * wq) @ V.T
    return Ahat, Mhat


def _kron_axes(mats):
    """Kronecker product with mats[a] acting on axis a (axis 0 fastest => rightmost factor)."""
    out = np.ones((1, 1))
    for a in reversed(range(len(mats))):
        out = np.kron(out, mats[a])
    return out


def cell_matrix(d, k, h):
    """Cell stiffness matrix on a Cartesian cell of side h (eq:mf with a diagonal Jacobian).

    A^K = sum_dir  (x)_{a} ( Ahat/h if a == dir else h*Mhat ), acting on the
    (k+1)^d cell DoFs numbered lexicographically with x0 fastest.
    """
    Ahat, Mhat = reference_matrices(k)
    total = 0.0
    for direction in range(d):
        mats = [Ahat / h if a == direction else h * Mhat for a in range(d)]
        total = total + _kron_axes(mats)
    return total


def cell_matrix_bruteforce(d, k, h):
    """Cell stiffness matrix from eq:matrix-def by d-dimensional quadrature, point by point.

    Used only to pin `cell_matrix`: loops over every tensor quadrature point and
    every pair of tensor-product basis functions, evaluating the full gradient.
    """
    g = gll_nodes(k)
    xq, wq = gauss_rule(k + 1)
    V = lagrange_values(g, xq)
    D = lagrange_derivatives(g, xq)
    nd = (k + 1) ** d
    A = np.zeros((nd, nd))
    local = list(itertools.product(range(k + 1), repeat=d))  # tuples (i_{d-1},...,i_0)
    for qidx in itertools.product(range(k + 1), repeat=d):
        w = np.prod([wq[q] for q in qidx]) * h ** d
        grads = np.zeros((nd, d))
        for n, multi in enumerate(local):
            # multi[-1-a] is the index along axis a; qidx likewise
            for a in range(d):
                val = 1.0
                for b in range(d):
                    i_b = multi[d - 1 - b]
                    q_b = qidx[d - 1 - b]
                    val *= (D[i_b, q_b] / h) if b == a else V[i_b, q_b]
                grads[n, a] = val
        A += w * grads @ grads.T
    return A
