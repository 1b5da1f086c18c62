// Shared device definitions: per-degree 1D tables in constant memory and
// launch-side helpers.  Each .hip translation unit holds its own copy of the
// constant tables and uploads it in its init function.
#pragma once
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace vps {

constexpr int kMaxN = 2 * kMaxDegree + 1;  // patch closure points per direction
constexpr int kMaxM = 2 * kMaxDegree - 1;  // patch interior points per direction

// Reciprocal eigenvalue sums of one degree (patch pair, reference cell size 1).  The colour pass
// indexes them by lane, so they live in constant memory; every other 1D table is a compile-time
// constant (generated header patch_tables_gen.hpp).
template <typename T>
struct DevTables {
  T inv3[kMaxM * kMaxM * kMaxM];  // 1 / (lam[a2] + lam[a1] + lam[a0]), index (a2*m + a1)*m + a0
  T inv2[kMaxM * kMaxM];          // 1 / (lam[a1] + lam[a0]),           index a1*m + a0
};

template <typename T>
inline void fill_dev_tables(int k, DevTables<T>& out) {
  const Tables1D& t = tables_for_degree(k);
  const int m = 2 * k - 1;
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
