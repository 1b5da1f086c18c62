// Host-side 1D tables of the Q_k vertex-patch method (reference cell [0,1]).
//
// Everything the kernels need is one-dimensional (Sec. 2.4: only 1D
// eigenvectors and eigenvalues are stored; Sec. 2.3: 1D shape data):
//   * Gauss-Lobatto support points (Sec. 2) and Gauss quadrature,
//   * reference stiffness Ahat and mass Mhat (eq:matrix-def on one cell),
//   * the two-cell patch matrices, interior rows x closure columns, which give
//     the Kronecker form of Abar_j (eq:tensorproduct_2d/3d),
//   * the generalised eigenpairs A S = M S Lambda, S^T M S = I of the
//     patch-interior 1D pair (eq:fast_inverse),
//   * band rows of the assembled 1D matrices (global operator, Sec. 2.3),
//   * prolongation coefficients (coarse Lagrange basis at fine nodes, Sec. 2.1)
//     and the restriction bands (their transpose).
// All tables are computed for h = 1; level scaling is applied by the kernels:
// Abar_h = h^(d-2) Abar_1 and A_j,h^{-1} = h^(2-d) A_j,1^{-1}.
#pragma once
#include <vector>

namespace vps {

constexpr int kMaxDegree = 7;

struct Tables1D {
  int k = 0;
  std::vector<double> gll;        // k+1 nodes
  std::vector<double> Ahat, Mhat; // (k+1)^2, row-major
  std::vector<double> Ac, Mc;     // patch: m x n (interior rows 1..2k-1, closure cols 0..2k), n=2k+1, m=2k-1
  std::vector<double> S;          // m x m, column j is eigenvector j: S[i*m + j]
  std::vector<double> lam;        // m
  std::vector<double> Aband, Mband;  // k x (2k+1): row of the assembled 1D matrix for node class c
  std::vector<double> P;          // (2k+1) x (k+1): phi_a at fine position q of a coarse cell
  std::vector<double> Rband;      // k x (4k+1): restriction row of coarse node class a over fine nodes
  std::vector<double> gauss_x, gauss_w;  // k+1 Gauss points / weights on [0,1]
};

// Build (or fetch from a process-wide cache) the tables of degree k (1..kMaxDegree).
const Tables1D& tables_for_degree(int k);

// Building blocks, exposed for tests.
void gauss_lobatto(int k, std::vector<double>& nodes);
void gauss_legendre(int nq, std::vector<double>& x, std::vector<double>& w);
double lagrange(const std::vector<double>& nodes, int i, double x);
double lagrange_deriv(const std::vector<double>& nodes, int i, double x);
// Generalised symmetric-definite eigenproblem A S = M S diag(lam), S^T M S = I (n x n row-major).
bool generalized_eigen(int n, const std::vector<double>& A, const std::vector<double>& M,
                       std::vector<double>& S, std::vector<double>& lam);

}  // namespace vps
