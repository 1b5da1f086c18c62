"""Plain FP64 CPU oracle for the vertex-patch multigrid method (test infrastructure).

This package is test infrastructure, not part of the product.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.
It shares no code with the HIP library: every formula here is written out from
the paper (arXiv 2405.19004) in the most direct form available -- explicit
Lagrange polynomials, explicitly assembled matrices, dense LU patch solves -- so
that it can be checked against the paper by eye.

Modules
  basis      1D support points, quadrature, Lagrange basis, reference matrices
             (Sec. 2, eq:weak_form / eq:matrix-def; Sec. 2.3 eq:mf)
  mesh       uniform level meshes, lexicographic DoFs, global operator,
             vertex patches and their colours (Sec. 2, Sec. 2.2, Fig. 2)
  smoother   patch matrices, dense-LU local solves, additive and colourised
             multiplicative Schwarz smoothers (Sec. 2.2, Alg. 3, eq:local-solver)
  fastdiag   fast-diagonalisation inverse used only as a cross-check
             (Sec. 2.4, eq:inverse2d/3d, eq:fast_inverse)
  transfer   prolongation by embedding and restriction as its transpose
             (Sec. 2.1)
  multigrid  coarse solve, V-cycle (Alg. 1), full multigrid (Alg. 2), PCG
  rhs        load vectors of separable sine right-hand sides and L2 errors

Conventions (the readings of the paper taken here)
  * level l has 2**l cells per direction, h = 2**-l, n1d = k*2**l + 1 nodes per
    direction; level 1 is the coarsest level and is solved exactly.
  * vectors are full-grid, lexicographic with x0 fastest (numpy C order of an
    array shaped (n1d,)*d read as [x_{d-1}, ..., x_0]); boundary entries are 0.
  * support points are Gauss-Lobatto points; all integrals use (k+1)-point
    Gauss-Legendre quadrature per cell direction.
  * vertex patch colours: c(v) = sum_i ((v_i - 1) mod 2) * 2**i.

Every function is FP64.  Nothing here is tuned for speed beyond using library
primitives (sparse products, LU) for the steps the paper defines.
"""
