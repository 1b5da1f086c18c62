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

// s + c x for a coefficient c that is a compile-time table entry.  IEEE arithmetic does not let the
// compiler drop fma(0, x, s) (x could be infinite), so a structural zero of a table would still cost
// a multiply-add; here it costs nothing, and for finite x the result is the same bit for bit.
// Only use it where c folds to a constant: otherwise the test becomes a select.
template <typename T>
__device__ __forceinline__ T fma_tab(T c, T x, T s) {
  return c == T(0) ? s : fma(c, x, s);
}

// Global access to p at a per-lane byte offset below 4 GiB, p wave-uniform: the load unit adds the
// 32-bit offset to the scalar base, so the lane needs no 64-bit address arithmetic.  p is pinned in
// scalar registers: the optimiser would otherwise fold the lane offset into one 64-bit per-lane
// address and add every other uniform base to it lane by lane.  (p must be uniform where it is
// computed: not a value defined inside a loop whose exit differs between lanes.)
#define VPS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ld_lane(const T* p, unsigned off) {
  const VPS_GLOBAL char* g = (const VPS_GLOBAL char*)p;
  asm volatile("" : "+s"(g));
  return *(const VPS_GLOBAL T*)(g + off);
}
template <typename T>
__device__ __forceinline__ void st_lane(T* p, unsigned off, T v) {
  VPS_GLOBAL char* g = (VPS_GLOBAL char*)p;
  asm volatile("" : "+s"(g));
  *(VPS_GLOBAL T*)(g + off) = v;
}

// Geometry of one level as the kernels see it.
struct LevelGeom {
  int dim, k, level;
  long long n1d;     // nodes per direction
  long long ncells;  // cells per direction (2^level)
  double h;
};

// Workgroup `blk` of a colour pass: PPW patches consecutive along x0 inside the colour whose patch
// grid is described by the vertex parities p[], the patch counts cnt0, cnt1 (and the third axis in
// 3D) and the workgroups per x0 row groups0.  The kernels and the host-side launch check both take
// the mapping from here.  s0..s2: closure corner of the first patch (node indices); first: index of
// that patch along x0 inside the colour; count: patches of the workgroup (1..PPW).
struct ColourBlock {
  long long s0, s1, s2;
  int first, count;
};
template <int D, int K, int PPW>
__host__ __device__ inline ColourBlock colour_block(unsigned blk, int p0, int p1, int p2, int cnt0, int cnt1,
                                                    int groups0) {
  const int g0 = blk % groups0;
  const int rest = blk / groups0;
  const int t1 = rest % cnt1;
  const int t2 = D == 3 ? rest / cnt1 : 0;
  ColourBlock cb;
  cb.first = g0 * PPW;
  cb.count = cnt0 - cb.first < PPW ? cnt0 - cb.first : PPW;
  cb.s0 = (long long)K * (p0 + 2 * cb.first);
  cb.s1 = (long long)K * (p1 + 2 * t1);
  cb.s2 = D == 3 ? (long long)K * (p2 + 2 * t2) : 0;
  return cb;
}

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
