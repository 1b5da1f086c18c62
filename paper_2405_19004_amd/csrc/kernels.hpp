// Launch functions of the device code (HIP translation units), called by the
// host-side library.  All launches are asynchronous on the given stream and
// return the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "device_common.hpp"

namespace vps {

// Scalar slots of the CG scalar block (device memory, doubles).
enum : int {
  kScRZ = 0,     // r.z of the current iterate
  kScPQ = 10,    // p.A p                         (written together with slot 11)
  kScRR = 2,     // r.r after the update          (written together with kScRZOld)
  kScRZOld = 3,  // r_new . z_old (flexible beta)
  kScRZNew = 4,  // r_new . z_new                 (written together with kScAux)
  kScAux = 5,
  kScBeta = 6,
  kScBB = 7,     // b.b
  kScTrue = 8,   // true residual norm squared    (written together with kScAux2)
  kScAux2 = 9,
  kScCount = 16
};

hipError_t init_smoother_tables();

// Colour-pass kernels: multiplicative (residual, then x^I += A_j^{-1} r), additive
// (x^I += A_j^{-1} b^I) and Boundary (x^I = A_j^{-1} (b^I - A^{IB} x^B), x^I never read).
// kModeMfma: the multiplicative pass with the residual contractions on the matrix cores (3D Q4
// FP32, default launch shape); elsewhere the same as kModeMultiplicative.
// kModeZero: colour 0 of the multiplicative pass on a zero iterate, x <- S_0(0, b): writes
// A_j^{-1} b^I on the colour's patch interiors and 0 on every other node (the closures of colour 0
// tile the grid), so x need not be cleared first and is never read.
enum { kModeMultiplicative = 0, kModeAdditive = 1, kModeBoundary = 2, kModeMfma = 4, kModeZero = 5 };

// One member of a packed colour-pass launch (see launch_colour_pass_group).
struct ColourPassDesc {
  const void* b;
  void* x;
  long long n1d;
  int p[3];
  int cnt0, cnt1, groups0;
  int block_begin;
  double res_scale, sol_scale;
};
constexpr int kMaxGroup = 16;
struct ColourPassGroup {
  int n;
  ColourPassDesc e[kMaxGroup];
};
struct ColourPassMember {
  LevelGeom g;
  const void* b;
  void* x;
};
// Colour `colour` on every member (same dim, degree and precision; any levels) with one launch
// per kMaxGroup members.  Each member's arithmetic is exactly that of launch_colour_pass.
hipError_t launch_colour_pass_group(int dim, int k, int prec, int mode, int colour,
                                    const ColourPassMember* members, int n_members, hipStream_t st);

// smoother.hip
hipError_t launch_colour_pass(const LevelGeom& g, int prec, int mode, int colour, const void* b, void* x,
                              hipStream_t st);

// grid.hip (interior outputs only)
hipError_t launch_operator(const LevelGeom& g, int prec, const void* x, const void* b_or_null, void* y, hipStream_t st);
// Per-workgroup partial sums the two fused operator forms below take on level g (0: no fused
// form on that level).
long long fused_reduction_parts(const LevelGeom& g);
// q = A p in FP64 with out[0] = p.q summed in a fixed order from per-workgroup partials (at most
// max_parts of them); *fused = false (nothing launched) where that form is not available.
hipError_t launch_operator_pq(const LevelGeom& g, const double* p, double* q, double* part, long long max_parts,
                              double* out, hipStream_t st, bool* fused);
// out[0] = |b - A x|^2 (interior, FP64) summed in a fixed order from per-workgroup partials, the
// residual itself not stored; *fused = false (nothing launched) where that form is not available.
hipError_t launch_residual_norm2(const LevelGeom& g, const double* x, const double* b, double* part,
                                 long long max_parts, double* out, hipStream_t st, bool* fused);
// Restriction P^T of a fine-level vector (fine boundary entries ignored, coarse boundary written 0);
// t is scratch of restrict_scratch_elems(fine) elements (none in 2D: one kernel, no intermediate).
// A non-null xc_zero (a coarse-level vector) is set to 0 as well, which saves the V-cycle a fill
// launch per level.
hipError_t launch_restrict(const LevelGeom& fine, int prec, const void* rf, void* rc, void* t, hipStream_t st,
                           void* xc_zero = nullptr);
inline long long restrict_scratch_elems(int dim, int k, int fine_level) {
  const long long nf = (long long)k * (1LL << fine_level) + 1, nc = (long long)k * (1LL << (fine_level - 1)) + 1;
  return dim == 2 ? 0 : nf * nc * nc;
}
hipError_t launch_prolongate_add(const LevelGeom& fine, int prec, const void* e, void* xf, hipStream_t st);
// The allocation-free restriction's scratch: a static device array of noalloc_scratch_bytes()
// bytes per GPU.  noalloc_scratch() returns its device address on the current device (looked up
// once per device and kept).
// Host-side launch geometry of one level (no device work): every colour-pass workgroup of every
// colour and launch shape maps to patches of that colour inside the grid, covers each patch once
// and stays within the kernels' 32-bit offsets; every operator and transfer launch fits its
// launcher's limits.  False with a reason otherwise; *blocks adds the workgroups enumerated.
bool check_colour_launches(const LevelGeom& g, long long* blocks, std::string* why);
bool check_grid_launches(const LevelGeom& g, std::string* why);
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(void** out);
hipError_t launch_zero_boundary(const LevelGeom& g, int prec, void* y, hipStream_t st);
hipError_t launch_rhs_separable(const LevelGeom& g, int prec, int nterms, const double* G, const double* coef, void* b,
                                hipStream_t st);

// Partial sums (nparts doubles) of the squared L2 error, cellwise nq-point Gauss (see grid.hip).
hipError_t launch_l2_error(const LevelGeom& g, const double* x, const double* V, const double* wq, const double* S,
                           const double* uc, int nmodes, int nq, double* partial, int nparts, hipStream_t st);

// vector.hip
int reduction_parts();  // partial slots the reductions use (pairs: 2x this many doubles)
hipError_t launch_fill(int prec, void* x, long long n, double v, hipStream_t st);
// dst = (double)src, zero = 0 (n entries each)
hipError_t launch_widen_zero(const float* src, double* dst, double* zero, long long n, hipStream_t st);
hipError_t launch_cast(int from_prec, const void* src, void* dst, long long n, hipStream_t st);
// dst = interior of src, out = |dst|^2, *bad |= non-finite entries; optionally dst32 = (float)dst
// and zero = 0 over the same range
hipError_t launch_copy_interior_norm(int dim, long long n1d, const double* src, double* dst, double* partial,
                                     double* out, int* bad, hipStream_t st, float* dst32 = nullptr,
                                     double* zero = nullptr);
hipError_t launch_dot2(const double* a, const double* b, const double* c, const double* d, long long n,
                       double* partial, double* out, hipStream_t st);
// x += alpha p, r -= alpha q with alpha = rz / pq, partials of r.r and r.z, and r32 = (float) r
// when r32 != null.  z is the previous preconditioned residual: the FP32 z32 (widened exactly)
// when non-null, else the FP64 z.
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, const double* z, const float* z32,
                            long long n, double* sc, double* partial, float* r32, hipStream_t st);
// out[0] = r.z32 with z32 widened exactly (deterministic)
hipError_t launch_dot_rz32(const float* z32, const double* r, long long n, double* partial, double* out,
                           hipStream_t st);
hipError_t launch_cg_beta(double* sc, int flexible, hipStream_t st);
// p = z + beta p (z32 widened exactly when non-null, else z)
hipError_t launch_cg_direction(double* p, const double* z, const float* z32, long long n, const double* sc,
                               hipStream_t st);

}  // namespace vps
