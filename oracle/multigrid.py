"""Coarse solve, V-cycle, full multigrid and preconditioned CG (oracle, test infrastructure).

Paper passages: Alg. 1 (V-cycle: pre-smooth, residual, restrict, recurse from
zero, prolongate-add, post-smooth; exact solve on the coarsest level), Alg. 2
(full multigrid; iteration count = repetitions of the final while loop), Sec. 2.1
(one pre- and one post-smoothing step; the coarsest level is solved exactly by
one smoother step).  The Krylov solver is plain preconditioned CG (the paper uses
GMRES; CG is the method the workloads here ask for), with the V-cycle as
preconditioner; post-smoothing runs the colours in reverse so the V-cycle is
symmetric.
"""
import functools

import numpy as np
import scipy.linalg as sla

from . import mesh, smoother, transfer

COARSEST = 1


@functools.lru_cache(maxsize=None)
def _coarse_lu(d, k):
    return sla.lu_factor(mesh.operator_matrix(d, k, COARSEST).toarray())


def coarse_solve(d, k, b):
    """x = A_1^{-1} b on level 1 by dense LU of the explicit interior matrix."""
    inner = mesh.interior_ids(d, k, COARSEST)
    x = np.zeros(mesh.n1d(k, COARSEST) ** d)
    x[inner] = sla.lu_solve(_coarse_lu(d, k), np.asarray(b)[inner])
    return x


def vcycle(d, k, level, b, x, post_reverse=True):
    """One V-cycle on `level` (Alg. 1) with one pre- and one post-smoothing step.

    Pre-smoothing runs the colours in ascending order.  Post-smoothing runs them
    in descending order when `post_reverse` (the V-cycle is then a symmetric
    operator, as CG needs) or ascending otherwise (Alg. 1 read literally: the
    same S_l before and after the coarse-grid correction).
    """
    if level == COARSEST:
        return coarse_solve(d, k, b)
    x = smoother.multiplicative(d, k, level, b, x, reverse=False)
    r = np.asarray(b) - mesh.apply_operator(d, k, level, x)
    rc = transfer.restrict(d, k, level, r)
    ec = vcycle(d, k, level - 1, rc, np.zeros_like(rc), post_reverse)
    x = x + transfer.prolongate(d, k, level, ec)
    return smoother.multiplicative(d, k, level, b, x, reverse=post_reverse)


def fmg(d, k, L, b_levels, eps, maxit=50, post_reverse=False):
    """Full multigrid (Alg. 2).  b_levels[l] is the right-hand side on level l (l = 1..L).

    Returns (x_L, n) where n counts repetitions of the final while loop.  The
    V-cycles use the literal Alg. 1 (same colour order before and after) unless
    `post_reverse` is set.
    """
    x = coarse_solve(d, k, b_levels[COARSEST])
    for level in range(COARSEST + 1, L + 1):
        x = transfer.prolongate(d, k, level, x)
        x = vcycle(d, k, level, b_levels[level], x, post_reverse)
    delta0 = np.linalg.norm(b_levels[L])
    delta = np.linalg.norm(b_levels[L] - mesh.apply_operator(d, k, L, x))
    n = 0
    while delta > eps * delta0 and n < maxit:
        x = vcycle(d, k, L, b_levels[L], x, post_reverse)
        delta = np.linalg.norm(b_levels[L] - mesh.apply_operator(d, k, L, x))
        n += 1
    return x, n


def pcg(d, k, L, b, rtol, maxit=100, precondition=True, flexible=False, post_reverse=True):
    """Preconditioned CG for A_L x = b from x0 = 0, one V-cycle as preconditioner.

    Stops when the recursively updated residual satisfies ||r||_2 <= rtol ||b||_2.
    `post_reverse` picks the colour order of the V-cycle's post-smoothing (see vcycle).
    With `flexible` the new direction takes the Polak-Ribiere coefficient
    beta = r_{k+1}.(z_{k+1} - z_k) / (r_k.z_k), which keeps CG convergent when the
    preconditioner is not a fixed symmetric operator (the literal colour order of Alg. 1, or
    an FP32 V-cycle inside the FP64 iteration); for a symmetric preconditioner r_{k+1}.z_k
    vanishes in exact arithmetic and the two coefficients agree.
    Returns (x, iterations, history of ||r||/||b||).
    """
    b = np.asarray(b, dtype=np.float64).copy()
    b[mesh.boundary_mask(d, k, L)] = 0.0
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist

    def prec(v):
        return vcycle(d, k, L, v, np.zeros_like(v), post_reverse) if precondition else v.copy()

    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = mesh.apply_operator(d, k, L, p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rtol:
            break
        z_new = prec(r)
        rz_new = r @ z_new
        beta = (rz_new - r @ z) / rz if flexible else rz_new / rz
        p = z_new + beta * p
        z, rz = z_new, rz_new
    return x, it, hist
