// Vector operations of the outer CG and the V-cycle (Sec. 3: element-wise and
// reduction-type vector operations).  Reductions are deterministic: a fixed
// grid writes one partial per workgroup (fixed in-group tree order) and a
// single workgroup sums the partials in a fixed order, so a result does not
// depend on scheduling.  CG scalars live in device memory; only the residual
// norm is copied to the host for the stopping test.
#include "device_common.hpp"
#include "kernels.hpp"

namespace vps {

namespace {

constexpr int kRedThreads = 256;
// Non-temporal loads and stores (the nt bit) for CG vector data that the next kernels do not read:
// they do not displace data the V-cycle and the operator reuse from the caches.  Used by the CG
// update: 3D Q4 64^3 mixed solve -3.1%, FP64 -1.5%, 2D Q7 512^2 -2.4% (the r.z product and the
// direction update, whose data the next kernel reads, measured slightly slower with them).
#ifndef VPS_CG_NT
#define VPS_CG_NT 1
#endif
// The CG set-up (copy_interior_kernel) likewise: b read, r and x = 0 written non-temporally (its
// FP32 residual feeds the first V-cycle): 3D Q4 64^3 mixed solve -0.7%, 2D Q7 512^2 -0.6%.
#ifndef VPS_SETUP_NT
#define VPS_SETUP_NT 1
#endif
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  if constexpr (VPS_CG_NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <typename T>
__device__ __forceinline__ void st_nt(T v, T* p) {
  if constexpr (VPS_CG_NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
// The dot-product loops take kUnroll strided elements per step: every load of the step is issued
// before the first use, and the elements are then summed in the order of the plain loop (same
// sums).  The CG update and the direction update measured no faster (slower) that way.
constexpr int kUnroll = 4;

template <typename T>
__global__ void fill_kernel(T* __restrict__ x, long long n, T v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

template <typename S, typename D>
__global__ void cast_kernel(const S* __restrict__ src, D* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// dst = (double)src and zero = 0 over the same range (the FP64 coarse solve of the FP32 V-cycle:
// its right-hand side and starting iterate in one launch)
__global__ void widen_zero_kernel(const float* __restrict__ src, double* __restrict__ dst, double* __restrict__ zero,
                                  long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    dst[i] = (double)src[i];
    zero[i] = 0.0;
  }
}

// dst = src with boundary entries 0 (FP64), also returns partials of src.src on the interior
// and a non-finite flag; optionally dst32 = dst rounded to FP32 and zero = 0 over the same range
// (the CG set-up: residual, its FP32 copy and the iterate in one pass).  I = unsigned int when
// every index fits in 32 bits (the coordinates then take 32-bit divisions), else long long.
template <typename I>
__global__ void copy_interior_kernel(const double* __restrict__ src, double* __restrict__ dst, int dim, long long n1d_,
                                     long long ntot_, double* __restrict__ partial, int* __restrict__ bad,
                                     float* __restrict__ dst32, double* __restrict__ zero) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  int nonfinite = 0;
  const I n1d = (I)n1d_, ntot = (I)ntot_;
  for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += (I)gridDim.x * blockDim.x) {
    const I i0 = i % n1d, r = i / n1d, i1 = r % n1d, i2 = r / n1d;
    bool bnd = i0 == 0 || i0 == n1d - 1 || i1 == 0 || i1 == n1d - 1 || (dim == 3 && (i2 == 0 || i2 == n1d - 1));
    double v = bnd ? 0.0 : (VPS_SETUP_NT ? __builtin_nontemporal_load(&src[i]) : src[i]);
    if (!isfinite(v)) nonfinite = 1;
    if constexpr (VPS_SETUP_NT) {
      __builtin_nontemporal_store(v, &dst[i]);
    } else {
      dst[i] = v;
    }
    if (dst32) dst32[i] = (float)v;
    if (zero) {
      if constexpr (VPS_SETUP_NT) {
        __builtin_nontemporal_store(0.0, &zero[i]);
      } else {
        zero[i] = 0.0;
      }
    }
    acc = fma(v, v, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  if (nonfinite) atomicOr(bad, 1);
}

__device__ __forceinline__ void block_reduce2(double a, double b, double* out_a, double* out_b) {
  __shared__ double ra[kRedThreads], rb[kRedThreads];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      ra[threadIdx.x] += ra[threadIdx.x + s];
      rb[threadIdx.x] += rb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out_a = ra[0];
    *out_b = rb[0];
  }
}

// partials of a.b (slot 0) and c.d (slot 1); c may be null
__global__ void dot2_kernel(const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ c,
                            const double* __restrict__ d, long long n, double* __restrict__ partial) {
  double s0 = 0.0, s1 = 0.0;
  const long long G = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kUnroll - 1) * G < n; i += kUnroll * G) {
    double va[kUnroll], vb[kUnroll], vc[kUnroll], vd[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      va[u] = a[i + u * G];
      vb[u] = b[i + u * G];
      if (c) {
        vc[u] = c[i + u * G];
        vd[u] = d[i + u * G];
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      s0 = fma(va[u], vb[u], s0);
      if (c) s1 = fma(vc[u], vd[u], s1);
    }
  }
  for (; i < n; i += G) {
    s0 = fma(a[i], b[i], s0);
    if (c) s1 = fma(c[i], d[i], s1);
  }
  block_reduce2(s0, s1, &partial[2 * blockIdx.x], &partial[2 * blockIdx.x + 1]);
}

// Sum 2*nparts partials (pairs) into out[0], out[1] in a fixed order.
__global__ void finalize2_kernel(const double* __restrict__ partial, int nparts, double* __restrict__ out) {
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    s0 += partial[2 * i];
    s1 += partial[2 * i + 1];
  }
  block_reduce2(s0, s1, &out[0], &out[1]);
}

__global__ void finalize1_kernel(const double* __restrict__ partial, int nparts, double* __restrict__ out) {
  double s0 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s0 += partial[i];
  double dummy;
  block_reduce2(s0, 0.0, &out[0], &dummy);
}

// CG step: x += alpha p, r -= alpha q, alpha = s[RZ] / s[PQ]; partials
// of r.r (slot 0) and r.z (slot 1, z = the previous preconditioned residual, FP64 or the FP32
// output of the FP32 preconditioner, widened exactly).  With r32 != null the updated residual is
// also stored rounded to FP32 (the input of the FP32 preconditioner), which saves a separate cast
// pass.
template <typename Z>
__global__ void cg_update_kernel(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                                 const double* __restrict__ q, const Z* __restrict__ z, long long n,
                                 const double* __restrict__ sc, double* __restrict__ partial, float* __restrict__ r32) {
  const double alpha = sc[kScRZ] / sc[kScPQ];
  double s0 = 0.0, s1 = 0.0;
  // x, r, p, q and z are next read after a V-cycle or never: non-temporal; r32 feeds the V-cycle
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    st_nt(fma(alpha, ld_nt(&p[i]), ld_nt(&x[i])), &x[i]);
    const double ri = fma(-alpha, ld_nt(&q[i]), ld_nt(&r[i]));
    st_nt(ri, &r[i]);
    if (r32) r32[i] = (float)ri;
    s0 = fma(ri, ri, s0);
    s1 = fma(ri, (double)ld_nt(&z[i]), s1);
  }
  block_reduce2(s0, s1, &partial[2 * blockIdx.x], &partial[2 * blockIdx.x + 1]);
}

// partials of r.z for the FP32 preconditioner output z32 (widened exactly): the FP64 copy of z is
// never stored, its consumers widen z32 as they read it.
__global__ void dot_rz32_kernel(const float* __restrict__ z32, const double* __restrict__ r, long long n,
                                double* __restrict__ partial) {
  double s0 = 0.0;
  const long long G = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kUnroll - 1) * G < n; i += kUnroll * G) {
    double vr[kUnroll];
    float vz[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      vr[u] = r[i + u * G];
      vz[u] = z32[i + u * G];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s0 = fma(vr[u], (double)vz[u], s0);
  }
  for (; i < n; i += G) s0 = fma(r[i], (double)z32[i], s0);
  block_reduce2(s0, 0.0, &partial[2 * blockIdx.x], &partial[2 * blockIdx.x + 1]);
}

// p = z + beta p, beta from the scalar block (z FP64, or FP32 widened exactly)
template <typename Z>
__global__ void cg_direction_kernel(double* __restrict__ p, const Z* __restrict__ z, long long n,
                                    const double* __restrict__ sc) {
  const double beta = sc[kScBeta];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = fma(beta, p[i], (double)z[i]);
}

// beta = (rz_new - flexible * r_new.z_old) / rz ; rz <- rz_new.  Also flags non-finite values.
__global__ void cg_beta_kernel(double* __restrict__ sc, int flexible) {
  const double rz_new = sc[kScRZNew];
  const double num = flexible ? rz_new - sc[kScRZOld] : rz_new;
  sc[kScBeta] = num / sc[kScRZ];
  sc[kScRZ] = rz_new;
}

}  // namespace

static unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

int reduction_parts() { return 1024; }

hipError_t launch_fill(int prec, void* x, long long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, (double*)x, n, v);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, (float*)x, n, (float)v);
  return hipGetLastError();
}

hipError_t launch_cast(int from_prec, const void* src, void* dst, long long n, hipStream_t st) {
  if (from_prec == 0)
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(grid_for(n)), dim3(256), 0, st, (const double*)src,
                       (float*)dst, n);
  else
    hipLaunchKernelGGL((cast_kernel<float, double>), dim3(grid_for(n)), dim3(256), 0, st, (const float*)src,
                       (double*)dst, n);
  return hipGetLastError();
}

hipError_t launch_widen_zero(const float* src, double* dst, double* zero, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, zero, n);
  return hipGetLastError();
}

hipError_t launch_copy_interior_norm(int dim, long long n1d, const double* src, double* dst, double* partial,
                                     double* out, int* bad, hipStream_t st, float* dst32, double* zero) {
  long long ntot = dim == 2 ? n1d * n1d : n1d * n1d * n1d;
  const int parts = reduction_parts();
  // 32-bit indices need ntot plus one grid stride to stay below 2^32
  if (ntot + (long long)parts * kRedThreads < (1LL << 32))
    hipLaunchKernelGGL(copy_interior_kernel<unsigned>, dim3(parts), dim3(kRedThreads), 0, st, src, dst, dim, n1d, ntot,
                       partial, bad, dst32, zero);
  else
    hipLaunchKernelGGL(copy_interior_kernel<long long>, dim3(parts), dim3(kRedThreads), 0, st, src, dst, dim, n1d, ntot,
                       partial, bad, dst32, zero);
  hipLaunchKernelGGL(finalize1_kernel, dim3(1), dim3(kRedThreads), 0, st, partial, parts, out);
  return hipGetLastError();
}

hipError_t launch_dot2(const double* a, const double* b, const double* c, const double* d, long long n,
                       double* partial, double* out, hipStream_t st) {
  const int parts = reduction_parts();
  hipLaunchKernelGGL(dot2_kernel, dim3(parts), dim3(kRedThreads), 0, st, a, b, c, d, n, partial);
  hipLaunchKernelGGL(finalize2_kernel, dim3(1), dim3(kRedThreads), 0, st, partial, parts, out);
  return hipGetLastError();
}

hipError_t launch_dot_rz32(const float* z32, const double* r, long long n, double* partial, double* out,
                           hipStream_t st) {
  const int parts = reduction_parts();
  hipLaunchKernelGGL(dot_rz32_kernel, dim3(parts), dim3(kRedThreads), 0, st, z32, r, n, partial);
  hipLaunchKernelGGL(finalize2_kernel, dim3(1), dim3(kRedThreads), 0, st, partial, parts, out);
  return hipGetLastError();
}

hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, const double* z, const float* z32,
                            long long n, double* sc, double* partial, float* r32, hipStream_t st) {
  const int parts = reduction_parts();
  if (z32)
    hipLaunchKernelGGL(cg_update_kernel<float>, dim3(parts), dim3(kRedThreads), 0, st, x, r, p, q, z32, n, sc, partial,
                       r32);
  else
    hipLaunchKernelGGL(cg_update_kernel<double>, dim3(parts), dim3(kRedThreads), 0, st, x, r, p, q, z, n, sc, partial,
                       r32);
  hipLaunchKernelGGL(finalize2_kernel, dim3(1), dim3(kRedThreads), 0, st, partial, parts, sc + kScRR);
  return hipGetLastError();
}

hipError_t launch_cg_beta(double* sc, int flexible, hipStream_t st) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(1), 0, st, sc, flexible);
  return hipGetLastError();
}

hipError_t launch_cg_direction(double* p, const double* z, const float* z32, long long n, const double* sc,
                               hipStream_t st) {
  if (z32)
    hipLaunchKernelGGL(cg_direction_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, p, z32, n, sc);
  else
    hipLaunchKernelGGL(cg_direction_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, p, z, n, sc);
  return hipGetLastError();
}

}  // namespace vps
