// Shared device definitions: per-degree 1D tables in constant memory and
// launch-side helpers.  Each .hip translation unit holds its own copy of the
// constant tables and uploads it in its init function.
#pragma once
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace vps {

constexpr int kMaxN = 2 * kMaxDegree + 1;  // patch closure points per direction
constexpr int kMaxM = 2 * kMaxDegree - 1;  // patch interior points per direction

// 1D tables of one degree, reference cell size 1 (see tables.hpp for meanings).
template <typename T>
struct DevTables {
  T Mc[kMaxM * kMaxN];  // patch mass, interior rows x closure cols (m x n)
  T Ac[kMaxM * kMaxN];  // patch stiffness, same shape
  T S[kMaxM * kMaxM];   // eigenvectors, S[i*m + a]
  T lam[kMaxM];         // eigenvalues
  T Mb[kMaxDegree * kMaxN];  // assembled-mass band rows, k x (2k+1)
  T Ab[kMaxDegree * kMaxN];  // assembled-stiffness band rows
  T P[kMaxN * (kMaxDegree + 1)];          // prolongation (2k+1) x (k+1)
  T Rb[kMaxDegree * (4 * kMaxDegree + 1)];  // restriction band rows k x (4k+1)
  T inv3[kMaxM * kMaxM * kMaxM];  // 1 / (lam[a2] + lam[a1] + lam[a0]), index (a2*m + a1)*m + a0
  T inv2[kMaxM * kMaxM];          // 1 / (lam[a1] + lam[a0]),           index a1*m + a0
  T Ah[(kMaxDegree + 1) * (kMaxDegree + 1)];  // reference cell stiffness (k+1) x (k+1)
  T Mh[(kMaxDegree + 1) * (kMaxDegree + 1)];  // reference cell mass
};

template <typename T>
inline void fill_dev_tables(int k, DevTables<T>& out) {
  const Tables1D& t = tables_for_degree(k);
  const int n = 2 * k + 1, m = 2 * k - 1, np = k + 1;
  for (int i = 0; i < m * n; ++i) { out.Mc[i] = (T)t.Mc[i]; out.Ac[i] = (T)t.Ac[i]; }
  for (int i = 0; i < m * m; ++i) out.S[i] = (T)t.S[i];
  for (int i = 0; i < m; ++i) out.lam[i] = (T)t.lam[i];
  for (int i = 0; i < k * n; ++i) { out.Mb[i] = (T)t.Mband[i]; out.Ab[i] = (T)t.Aband[i]; }
  for (int i = 0; i < n * np; ++i) out.P[i] = (T)t.P[i];
  for (int i = 0; i < k * (4 * k + 1); ++i) out.Rb[i] = (T)t.Rband[i];
  for (int i = 0; i < np * np; ++i) { out.Ah[i] = (T)t.Ahat[i]; out.Mh[i] = (T)t.Mhat[i]; }
  for (int a2 = 0; a2 < m; ++a2)
    for (int a1 = 0; a1 < m; ++a1) {
      out.inv2[a2 * m + a1] = (T)(1.0 / (t.lam[a2] + t.lam[a1]));
      for (int a0 = 0; a0 < m; ++a0) out.inv3[(a2 * m + a1) * m + a0] = (T)(1.0 / (t.lam[a2] + t.lam[a1] + t.lam[a0]));
    }
}

// Geometry of one level as the kernels see it.
struct LevelGeom {
  int dim, k, level;
  long long n1d;     // nodes per direction
  long long ncells;  // cells per direction (2^level)
  double h;
};

// Round-robin XCD dispatch on MI355X: consecutive workgroup ids land on
// consecutive XCDs (8 of them).  Remap so that each XCD receives a contiguous
// run of logical tiles, which keeps neighbouring tiles (sharing faces) in the
// same L2.  Valid for any grid size: ids beyond the last full round keep their
// identity.
__device__ inline unsigned xcd_remap(unsigned bid, unsigned nblocks) {
  constexpr unsigned kXcd = 8;
  unsigned full = (nblocks / kXcd) * kXcd;
  if (bid >= full) return bid;
  unsigned per = full / kXcd;
  return (bid % kXcd) * per + bid / kXcd;
}

inline hipError_t upload_symbol(const void* symbol, const void* src, size_t bytes) {
  return hipMemcpyToSymbol(symbol, src, bytes, 0, hipMemcpyHostToDevice);
}

}  // namespace vps
