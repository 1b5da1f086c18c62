// Host-side 1D tables (see tables.hpp).  Written from the mathematics: Newton
// iterations for the Gauss and Gauss-Lobatto points, product-form Lagrange
// polynomials, Cholesky + cyclic Jacobi for the generalised eigenproblem.
#include "tables.hpp"

#include <cmath>
#include <mutex>
#include <stdexcept>

namespace vps {

namespace {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 1; j < n; ++j) {
    double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // (x^2 - 1) P_n' = n (x P_n - P_{n-1})
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

}  // namespace

void gauss_legendre(int nq, std::vector<double>& x, std::vector<double>& w) {
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  const double pi = std::acos(-1.0);
  for (int i = 0; i < nq; ++i) {
    double t = std::cos(pi * (i + 0.75) / (nq + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(nq, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    double p, dp;
    legendre(nq, t, p, dp);
    // map [-1,1] -> [0,1]; nodes ascending
    x[nq - 1 - i] = 0.5 * (t + 1.0);
    w[nq - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) halved
  }
}

void gauss_lobatto(int k, std::vector<double>& nodes) {
  // interior nodes: roots of P_k' ; P_k'' from the Legendre equation
  // (1 - t^2) P'' = 2 t P' - k(k+1) P.
  nodes.assign(k + 1, 0.0);
  nodes[0] = 0.0;
  nodes[k] = 1.0;
  const double pi = std::acos(-1.0);
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(pi * j / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, t, p, dp);
      double d2p = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    nodes[j] = 0.5 * (t + 1.0);
  }
}

double lagrange(const std::vector<double>& nodes, int i, double x) {
  double v = 1.0;
  for (size_t j = 0; j < nodes.size(); ++j)
    if ((int)j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
  return v;
}

double lagrange_deriv(const std::vector<double>& nodes, int i, double x) {
  double s = 0.0;
  for (size_t l = 0; l < nodes.size(); ++l) {
    if ((int)l == i) continue;
    double t = 1.0 / (nodes[i] - nodes[l]);
    for (size_t j = 0; j < nodes.size(); ++j)
      if ((int)j != i && j != l) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    s += t;
  }
  return s;
}

bool generalized_eigen(int n, const std::vector<double>& A, const std::vector<double>& M,
                       std::vector<double>& S, std::vector<double>& lam) {
  // M = L L^T (Cholesky)
  std::vector<double> L(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = M[i * n + j];
      for (int p = 0; p < j; ++p) s -= L[i * n + p] * L[j * n + p];
      if (i == j) {
        if (s <= 0.0) return false;
        L[i * n + i] = std::sqrt(s);
      } else {
        L[i * n + j] = s / L[j * n + j];
      }
    }
  }
  // C = L^{-1} A L^{-T}: first X = L^{-1} A (forward substitution per column), then C = X L^{-T}
  std::vector<double> X(n * n), C(n * n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = A[i * n + c];
      for (int p = 0; p < i; ++p) s -= L[i * n + p] * X[p * n + c];
      X[i * n + c] = s / L[i * n + i];
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double s = X[r * n + i];
      for (int p = 0; p < i; ++p) s -= C[r * n + p] * L[i * n + p];
      C[r * n + i] = s / L[i * n + i];
    }
  for (int i = 0; i < n; ++i)  // symmetrise rounding
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (C[i * n + j] + C[j * n + i]);
      C[i * n + j] = C[j * n + i] = s;
    }
  // cyclic Jacobi: C = Q diag Q^T
  std::vector<double> Q(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += C[i * n + j] * C[i * n + j];
        if (i != j) off += C[i * n + j] * C[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = C[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          double crp = C[r * n + p], crq = C[r * n + q];
          C[r * n + p] = c * crp - s * crq;
          C[r * n + q] = s * crp + c * crq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          double cpr = C[p * n + r], cqr = C[q * n + r];
          C[p * n + r] = c * cpr - s * cqr;
          C[q * n + r] = s * cpr + c * cqr;
        }
        for (int r = 0; r < n; ++r) {
          double qrp = Q[r * n + p], qrq = Q[r * n + q];
          Q[r * n + p] = c * qrp - s * qrq;
          Q[r * n + q] = s * qrp + c * qrq;
        }
      }
  }
  lam.assign(n, 0.0);
  for (int i = 0; i < n; ++i) lam[i] = C[i * n + i];
  // S = L^{-T} Q (back substitution per column)
  S.assign(n * n, 0.0);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[i * n + c];
      for (int p = i + 1; p < n; ++p) s -= L[p * n + i] * S[p * n + c];
      S[i * n + c] = s / L[i * n + i];
    }
  return true;
}

namespace {

Tables1D build(int k) {
  Tables1D t;
  t.k = k;
  gauss_lobatto(k, t.gll);
  gauss_legendre(k + 1, t.gauss_x, t.gauss_w);
  const int np = k + 1;
  t.Ahat.assign(np * np, 0.0);
  t.Mhat.assign(np * np, 0.0);
  for (int q = 0; q < np; ++q) {
    double xq = t.gauss_x[q], wq = t.gauss_w[q];
    for (int i = 0; i < np; ++i)
      for (int j = 0; j < np; ++j) {
        t.Ahat[i * np + j] += wq * lagrange_deriv(t.gll, i, xq) * lagrange_deriv(t.gll, j, xq);
        t.Mhat[i * np + j] += wq * lagrange(t.gll, i, xq) * lagrange(t.gll, j, xq);
      }
  }
  // two-cell patch closure matrices (n x n), unit cells
  const int n = 2 * k + 1, m = 2 * k - 1;
  std::vector<double> Apc(n * n, 0.0), Mpc(n * n, 0.0);
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < np; ++i)
      for (int j = 0; j < np; ++j) {
        Apc[(k * c + i) * n + k * c + j] += t.Ahat[i * np + j];
        Mpc[(k * c + i) * n + k * c + j] += t.Mhat[i * np + j];
      }
  t.Ac.assign(m * n, 0.0);
  t.Mc.assign(m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      t.Ac[i * n + j] = Apc[(i + 1) * n + j];
      t.Mc[i * n + j] = Mpc[(i + 1) * n + j];
    }
  std::vector<double> Ai(m * m), Mi(m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      Ai[i * m + j] = Apc[(i + 1) * n + j + 1];
      Mi[i * m + j] = Mpc[(i + 1) * n + j + 1];
    }
  if (!generalized_eigen(m, Ai, Mi, t.S, t.lam)) throw std::runtime_error("patch mass matrix not SPD");
  // band rows of the assembled 1D matrices: node class c = i mod k, band covers
  // columns i - c - k .. i - c + k.
  t.Aband.assign(k * n, 0.0);
  t.Mband.assign(k * n, 0.0);
  for (int c = 0; c < k; ++c) {
    if (c == 0) {
      for (int j = 0; j <= k; ++j) {  // left cell: local row k
        t.Aband[j] += t.Ahat[k * np + j];
        t.Mband[j] += t.Mhat[k * np + j];
      }
      for (int j = 0; j <= k; ++j) {  // right cell: local row 0
        t.Aband[k + j] += t.Ahat[0 * np + j];
        t.Mband[k + j] += t.Mhat[0 * np + j];
      }
    } else {
      for (int j = 0; j <= k; ++j) {
        t.Aband[c * n + k + j] = t.Ahat[c * np + j];
        t.Mband[c * n + k + j] = t.Mhat[c * np + j];
      }
    }
  }
  // prolongation: fine position q (0..2k) of a coarse cell sits at g_q/2 (q <= k) or 1/2 + g_{q-k}/2
  t.P.assign(n * np, 0.0);
  for (int q = 0; q < n; ++q) {
    double xq = q <= k ? 0.5 * t.gll[q] : 0.5 + 0.5 * t.gll[q - k];
    for (int a = 0; a < np; ++a) {
      double v = lagrange(t.gll, a, xq);
      if (q == 0) v = (a == 0) ? 1.0 : 0.0;
      if (q == 2 * k) v = (a == k) ? 1.0 : 0.0;
      if (q == k && (k % 2 == 0)) v = (a == k / 2) ? 1.0 : 0.0;  // midpoint is a GLL node for even k
      t.P[q * np + a] = v;
    }
  }
  // restriction band: coarse node class a, columns 2k(C-1) .. 2k(C+1) over fine nodes
  const int rb = 4 * k + 1;
  t.Rband.assign(k * rb, 0.0);
  for (int a = 0; a < k; ++a) {
    if (a == 0) {
      for (int q = 0; q <= 2 * k; ++q) t.Rband[q] += t.P[q * np + k];          // left coarse cell, local index k
      for (int q = 1; q <= 2 * k; ++q) t.Rband[2 * k + q] += t.P[q * np + 0];  // right coarse cell, local index 0
    } else {
      for (int q = 0; q <= 2 * k; ++q) t.Rband[a * rb + 2 * k + q] = t.P[q * np + a];
    }
  }
  return t;
}

}  // namespace

const Tables1D& tables_for_degree(int k) {
  static std::mutex mu;
  static Tables1D cache[kMaxDegree + 1];
  static bool built[kMaxDegree + 1] = {};
  if (k < 1 || k > kMaxDegree) throw std::invalid_argument("degree out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!built[k]) {
    cache[k] = build(k);
    built[k] = true;
  }
  return cache[k];
}

}  // namespace vps
