// Vertex-patch smoother colour pass for gfx950 (the hot kernel).
//
// One launch processes every patch of one colour (Alg. 3: colours are
// sequential, patches inside a colour are disjoint and run in parallel).  Per
// patch j, multiplicative mode computes
//   r_j = b_j^I - Abar_j x_j          localised residual (Sec. 2.2)
//   x_j^I += A_j^{-1} r_j             fast diagonalisation (eq:inverse2d/3d)
// where Abar_j = sum_dir (x) of 1D patch matrices (eq:tensorproduct_2d/3d) is
// applied by sum factorisation with the partial products reused across
// directions (Sec. 3.1.1), and A_j^{-1} = (S x..x S)(sum Lambda)^{-1}(S x..x S)^T.
// Additive mode skips the residual: x^I += A_j^{-1} b_j^I.
//
// Mapping (designed for CDNA4, not a translation of the paper's CUDA):
//  * a workgroup owns PPW patches that are consecutive along x0 inside the
//    colour; their closures tile one contiguous x0 segment of 2k*PPW+1 nodes,
//    so the closure load is one coalesced sweep over rows and shared faces are
//    read once;
//  * every 1D contraction is done by a thread that holds one whole line (a
//    1D fibre of the patch tensor) in registers and multiplies it by the 1D
//    matrix, whose entries are wave-uniform and come from constant memory
//    through the scalar cache (SGPR operands of v_fma);
//  * LDS only transposes between directions: one write and one read per value
//    per direction change, never one LDS read per multiply-add.
// No atomics: patches of one colour write disjoint interiors.
#include "device_common.hpp"
#include "kernels.hpp"

namespace vps {

static __constant__ DevTables<double> g_tab64[kMaxDegree + 1];
static __constant__ DevTables<float> g_tab32[kMaxDegree + 1];

template <typename T>
__device__ __forceinline__ const DevTables<T>& tab(int k);
template <>
__device__ __forceinline__ const DevTables<double>& tab<double>(int k) { return g_tab64[k]; }
template <>
__device__ __forceinline__ const DevTables<float>& tab<float>(int k) { return g_tab32[k]; }

// Launch shape per (dim, degree): patches per workgroup and threads.
template <int D, int K>
struct SmootherShape;
template <int K> struct SmootherShape<2, K> {
  static constexpr int PPW = K == 1 ? 64 : K == 2 ? 32 : K == 3 ? 16 : K <= 5 ? 12 : 8;
  static constexpr int NT = 128;
};
template <int K> struct SmootherShape<3, K> {
  static constexpr int PPW = K == 1 ? 32 : K == 2 ? 8 : K == 3 ? 4 : K == 4 ? 2 : 1;
  static constexpr int NT = K <= 4 ? 128 : K == 5 ? 128 : K == 6 ? 192 : 256;
};

template <int D, int K, typename T, bool ADD>
struct SmootherLds {
  static constexpr int n = 2 * K + 1, m = 2 * K - 1;
  static constexpr int PPW = SmootherShape<D, K>::PPW;
  static constexpr int RS = 2 * K * PPW + 1;  // closure row segment of the workgroup
  static constexpr int X = ADD ? 0 : (D == 3 ? n * n * RS : n * RS);
  static constexpr int A3 = ADD ? PPW * m * m * m : (2 * PPW * n * n * m > PPW * m * m * m ? 2 * PPW * n * n * m : PPW * m * m * m);
  static constexpr int B3 = ADD ? PPW * m * m * m : (2 * PPW * n * m * m > PPW * m * m * m ? 2 * PPW * n * m * m : PPW * m * m * m);
  static constexpr int A2 = ADD ? PPW * m * m : (2 * PPW * n * m > PPW * m * m ? 2 * PPW * n * m : PPW * m * m);
  static constexpr int B2 = PPW * m * m;
  static constexpr int BX3 = X > B3 ? X : B3;
  static constexpr int BX2 = X > B2 ? X : B2;
  static constexpr int total = D == 3 ? A3 + BX3 : A2 + BX2;
  static constexpr int offA = 0;
  static constexpr int offB = D == 3 ? A3 : A2;
};

// The constant tables re-derived through an opaque (but wave-uniform) zero
// offset: keeps the compiler from hoisting every table load out of a stage's
// task loop, which would pin more values in SGPRs than exist and spill them.
template <typename T>
__device__ __forceinline__ const DevTables<T>& tab_fresh(int k) {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return *reinterpret_cast<const DevTables<T>*>(reinterpret_cast<const char*>(&tab<T>(k)) + z);
}

template <int D, int K, typename T, bool ADD>
__global__ __launch_bounds__((SmootherShape<D, K>::NT)) void colour_pass_kernel(
    const T* __restrict__ b, T* __restrict__ x, long long n1d, int p0, int p1, int p2, int cnt0, int cnt1,
    int groups0, T res_scale, T sol_scale) {
  constexpr int n = 2 * K + 1, m = 2 * K - 1;
  constexpr int PPW = SmootherShape<D, K>::PPW, NT = SmootherShape<D, K>::NT;
  using L = SmootherLds<D, K, T, ADD>;
  constexpr int RS = L::RS;
  constexpr int RW = 2 * K * PPW;  // interior row segment incl. the shared-face gaps
  __shared__ T smem[L::total];
  T* bufA = smem + L::offA;
  T* bufB = smem + L::offB;

  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int g0 = blk % groups0;
  const int rest = blk / groups0;
  const int t1 = rest % cnt1;
  const int t2 = D == 3 ? rest / cnt1 : 0;
  const int tfirst = g0 * PPW;
  const int P = min(PPW, cnt0 - tfirst);
  const long long s0 = (long long)K * (p0 + 2 * tfirst);
  const long long s1 = (long long)K * (p1 + 2 * t1);
  const long long s2 = D == 3 ? (long long)K * (p2 + 2 * t2) : 0;
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x;
  const int seg = 2 * K * P + 1;  // valid length of the closure row segment

  // rows of the patch-interior block handled by stage "b" (residual/Sᵀ along the slowest axis):
  // task = (i1, q, i0) in 3D, (q, i0) in 2D; prefetch b there before anything else.
  constexpr int NB = D == 3 ? PPW * m * m : PPW * m;
  constexpr int RB = (NB + NT - 1) / NT;
  // Offsets inside one workgroup's block fit in 32 bits (checked by the launcher).
  const int ld1 = (int)n1d, ld2 = D == 3 ? (int)n1d2 : 0;
  const long long origin = (D == 3 ? s2 * n1d2 : 0) + s1 * n1d + s0;  // closure corner of the first patch
  T* xo = x + origin;  // same restrict object as x: closure loads, x^I loads and stores
  const T* bo = b + origin;
  T bpre[RB][m];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    int q, i0, i1;
    if constexpr (D == 3) {
      i1 = task / (PPW * m);
      const int r = task - i1 * (PPW * m);
      q = r / m;
      i0 = r - q * m;
    } else {
      q = task / m;
      i0 = task - q * m;
      i1 = 0;
    }
    // clamp to a valid patch-interior position: the loads are then always in bounds and the
    // values of inactive tasks are simply never used
    q = min(q, P - 1);
    if constexpr (D == 3) i1 = min(i1, m - 1);
    const int off = (D == 3 ? ld2 + (1 + i1) * ld1 : ld1) + 2 * K * q + 1 + i0;
    const int st = D == 3 ? ld2 : ld1;
#pragma unroll
    for (int i = 0; i < m; ++i) bpre[rr][i] = bo[off + i * st];
  }

  // ---- closure segment -> LDS.  Work item = (column c, row j1 in 3D); the slowest axis is
  // walked in an unrolled loop, so an address costs one add and the Dirichlet tests on that
  // axis are compile-time.  Every closure node lies inside the grid: loads are unconditional
  // and Dirichlet nodes are replaced by 0 afterwards (boundary entries of x are ignored).
  if constexpr (!ADD) {
    T* X = bufB;
    constexpr int NW = D == 3 ? RS * n : RS;
    const bool lo1 = s1 == 0, hi1 = s1 + n - 1 == n1d - 1;
    const bool lo2 = D == 3 && s2 == 0, hi2 = D == 3 && s2 + n - 1 == n1d - 1;
    for (int w = tid; w < NW; w += NT) {
      const int c = w % RS, j1 = D == 3 ? w / RS : 0;
      const int cl = min(c, seg - 1);
      const long long gc = s0 + cl;
      bool bad = gc == 0 || gc == n1d - 1;
      if constexpr (D == 3) bad = bad || (j1 == 0 && lo1) || (j1 == n - 1 && hi1);
      const int base = (D == 3 ? j1 * ld1 : 0) + cl;
      constexpr int NS = n;  // slow-axis length (j2 in 3D, j1 in 2D)
      const int sstride = D == 3 ? ld2 : ld1;
      T v[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) v[j] = xo[base + j * sstride];
      const bool lo = D == 3 ? lo2 : lo1, hi = D == 3 ? hi2 : hi1;
      if (c < seg) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          const bool zero = bad || (j == 0 && lo) || (j == NS - 1 && hi);
          X[(D == 3 ? j * n + j1 : j) * RS + c] = zero ? T(0) : v[j];
        }
      }
    }
    __syncthreads();
  }

  if constexpr (D == 3) {
    T* U = bufB;  // [q][j2][i1][i0]
    T* V = bufB + PPW * n * m * m;
    if constexpr (!ADD) {
      const T* X = bufB;
      T* PM = bufA;
      T* PA = bufA + PPW * n * n * m;
      // ---- contract x0 with Mc and Ac: lines (q, j2, j1) of n values
      for (int base = 0; base < PPW * n * n; base += NT) {
        const int task = base + tid;
        const int q = task / (n * n), r = task - q * (n * n);
        if (task < PPW * n * n && q < P) {
          const DevTables<T>& tb = tab_fresh<T>(K);
          T in[n];
#pragma unroll
          for (int j = 0; j < n; ++j) in[j] = X[r * RS + 2 * K * q + j];
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sm = fma(tb.Mc[i * n + j], in[j], sm);
            PM[(q * n * n + r) * m + i] = sm;
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sa = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sa = fma(tb.Ac[i * n + j], in[j], sa);
            PA[(q * n * n + r) * m + i] = sa;
          }
        }
      }
      __syncthreads();
      // ---- contract x1: lines (q, j2, i0) along j1; U = M1 (M0 x), V = A1 (M0 x) + M1 (A0 x)
      for (int base = 0; base < PPW * n * m; base += NT) {
        const int task = base + tid;
        const int q = task / (n * m), r = task - q * (n * m);
        const int j2 = r / m, i0 = r - j2 * m;
        if (task < PPW * n * m && q < P) {
          const DevTables<T>& tb = tab_fresh<T>(K);
          T pm[n], pa[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            pm[j] = PM[((q * n + j2) * n + j) * m + i0];
            pa[j] = PA[((q * n + j2) * n + j) * m + i0];
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T su = T(0), sv = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              su = fma(tb.Mc[i * n + j], pm[j], su);
              sv = fma(tb.Ac[i * n + j], pm[j], sv);
              sv = fma(tb.Mc[i * n + j], pa[j], sv);
            }
            U[((q * n + j2) * m + i) * m + i0] = su;
            V[((q * n + j2) * m + i) * m + i0] = sv;
          }
        }
      }
      __syncthreads();
    }
    // ---- contract x2 (residual) and apply Sᵀ along x2: lines (i1, q, i0)
    T* W = bufA;  // [q][a2][i1][i0]
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int i1 = task / (PPW * m), r = task - i1 * (PPW * m);
      const int q = r / m, i0 = r - q * m;
      if (task < NB && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T res[m];
        if constexpr (ADD) {
#pragma unroll
          for (int i = 0; i < m; ++i) res[i] = bpre[rr][i];
        } else {
          T u[n], v[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            u[j] = U[((q * n + j) * m + i1) * m + i0];
            v[j] = V[((q * n + j) * m + i1) * m + i0];
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              s = fma(tb.Ac[i * n + j], u[j], s);
              s = fma(tb.Mc[i * n + j], v[j], s);
            }
            res[i] = fma(-res_scale, s, bpre[rr][i]);
          }
        }
#pragma unroll
        for (int a = 0; a < m; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < m; ++i) s = fma(tb.S[i * m + a], res[i], s);
          W[((q * m + a) * m + i1) * m + i0] = s;
        }
      }
    }
    __syncthreads();
    // ---- Sᵀ along x1: lines (q, a2, i0)
    T* W2 = bufB;
    for (int base = 0; base < PPW * m * m; base += NT) {
      const int task = base + tid;
      const int q = task / (m * m), r = task - q * (m * m);
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * m * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W[((q * m + a2) * m + i) * m + i0];
#pragma unroll
        for (int a = 0; a < m; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < m; ++i) s = fma(tb.S[i * m + a], in[i], s);
          W2[((q * m + a2) * m + a) * m + i0] = s;
        }
      }
    }
    __syncthreads();
    // ---- Sᵀ along x0, scale by 1/(lam2+lam1+lam0), S along x0: lines (q, a2, a1)
    for (int base = 0; base < PPW * m * m; base += NT) {
      const int task = base + tid;
      const int q = task / (m * m), r = task - q * (m * m);
      if (task < PPW * m * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m], z[m];
        const int basei = (q * m * m + r) * m;
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W2[basei + i];
#pragma unroll
        for (int a = 0; a < m; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < m; ++i) s = fma(tb.S[i * m + a], in[i], s);
          z[a] = s * tb.inv3[r * m + a];
        }
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < m; ++a) s = fma(tb.S[i * m + a], z[a], s);
          W[basei + i] = s;
        }
      }
    }
    __syncthreads();
    // ---- S along x1: lines (q, a2, i0)
    for (int base = 0; base < PPW * m * m; base += NT) {
      const int task = base + tid;
      const int q = task / (m * m), r = task - q * (m * m);
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * m * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W[((q * m + a2) * m + a) * m + i0];
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < m; ++a) s = fma(tb.S[i * m + a], in[a], s);
          W2[((q * m + a2) * m + i) * m + i0] = s;
        }
      }
    }
    __syncthreads();
    // ---- S along x2: lines (q, i1, i0); correction -> LDS [q][i2][i1][i0]
    for (int base = 0; base < PPW * m * m; base += NT) {
      const int task = base + tid;
      const int q = task / (m * m), r = task - q * (m * m);
      const int i1 = r / m, i0 = r - i1 * m;
      if (task < PPW * m * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W2[((q * m + a) * m + i1) * m + i0];
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < m; ++a) s = fma(tb.S[i * m + a], in[a], s);
          W[((q * m + i) * m + i1) * m + i0] = sol_scale * s;
        }
      }
    }
    __syncthreads();
    // ---- x^I += correction.  Work item = (column c, row i1); i2 walked unrolled; reads
    //      issued before writes.
    for (int w = tid; w < RW * m; w += NT) {
      const int c = w % RW, i1 = w / RW;
      const int q = c / (2 * K), i0 = c - q * (2 * K);
      if (q < P && i0 < m) {
        const int base = ld2 + (1 + i1) * ld1 + 1 + c;
        T old[m];
#pragma unroll
        for (int i2 = 0; i2 < m; ++i2) old[i2] = xo[base + i2 * ld2];
#pragma unroll
        for (int i2 = 0; i2 < m; ++i2) xo[base + i2 * ld2] = old[i2] + W[((q * m + i2) * m + i1) * m + i0];
      }
    }
  } else {
    // ================================ 2D =====================================
    T* W = bufB;  // [q][a1][i0]
    if constexpr (!ADD) {
      const T* X = bufB;
      T* PM = bufA;
      T* PA = bufA + PPW * n * m;
      // ---- contract x0 with Mc and Ac: lines (q, j1)
      for (int base = 0; base < PPW * n; base += NT) {
        const int task = base + tid;
        const int q = task / n, j1 = task - q * n;
        if (task < PPW * n && q < P) {
          const DevTables<T>& tb = tab_fresh<T>(K);
          T in[n];
#pragma unroll
          for (int j = 0; j < n; ++j) in[j] = X[j1 * RS + 2 * K * q + j];
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sm = fma(tb.Mc[i * n + j], in[j], sm);
            PM[(q * n + j1) * m + i] = sm;
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sa = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sa = fma(tb.Ac[i * n + j], in[j], sa);
            PA[(q * n + j1) * m + i] = sa;
          }
        }
      }
      __syncthreads();
    }
    // ---- residual along x1, r = b - (A1 (M0 x) + M1 (A0 x)) (or r = b), then Sᵀ along x1
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / m, i0 = task - q * m;
      if (task < NB && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T res[m];
        if constexpr (ADD) {
#pragma unroll
          for (int i = 0; i < m; ++i) res[i] = bpre[rr][i];
        } else {
          const T* PM = bufA;
          const T* PA = bufA + PPW * n * m;
          T pm[n], pa[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            pm[j] = PM[(q * n + j) * m + i0];
            pa[j] = PA[(q * n + j) * m + i0];
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              s = fma(tb.Ac[i * n + j], pm[j], s);
              s = fma(tb.Mc[i * n + j], pa[j], s);
            }
            res[i] = fma(-res_scale, s, bpre[rr][i]);
          }
        }
#pragma unroll
        for (int a = 0; a < m; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < m; ++i) s = fma(tb.S[i * m + a], res[i], s);
          W[(q * m + a) * m + i0] = s;
        }
      }
    }
    __syncthreads();
    // ---- Sᵀ along x0, scale by 1/(lam1+lam0), S along x0: lines (q, a1)
    T* W2 = bufA;
    for (int base = 0; base < PPW * m; base += NT) {
      const int task = base + tid;
      const int q = task / m, a1 = task - q * m;
      if (task < PPW * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m], z[m];
        const int basei = (q * m + a1) * m;
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W[basei + i];
#pragma unroll
        for (int a = 0; a < m; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < m; ++i) s = fma(tb.S[i * m + a], in[i], s);
          z[a] = s * tb.inv2[a1 * m + a];
        }
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < m; ++a) s = fma(tb.S[i * m + a], z[a], s);
          W2[basei + i] = s;
        }
      }
    }
    __syncthreads();
    // ---- S along x1: lines (q, i0); correction -> LDS [q][i1][i0]
    T* E = bufB;
    for (int base = 0; base < PPW * m; base += NT) {
      const int task = base + tid;
      const int q = task / m, i0 = task - q * m;
      if (task < PPW * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W2[(q * m + a) * m + i0];
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < m; ++a) s = fma(tb.S[i * m + a], in[a], s);
          E[(q * m + i) * m + i0] = sol_scale * s;
        }
      }
    }
    __syncthreads();
    // ---- x^I += correction.  Work item = column c; i1 walked unrolled; reads before writes.
    for (int c = tid; c < RW; c += NT) {
      const int q = c / (2 * K), i0 = c - q * (2 * K);
      if (q < P && i0 < m) {
        const int base = ld1 + 1 + c;
        T old[m];
#pragma unroll
        for (int i1 = 0; i1 < m; ++i1) old[i1] = xo[base + i1 * ld1];
#pragma unroll
        for (int i1 = 0; i1 < m; ++i1) xo[base + i1 * ld1] = old[i1] + E[(q * m + i1) * m + i0];
      }
    }
  }
}

// ------------------------------------------------------------------ host side

template <int D, int K, typename T, bool ADD>
static hipError_t launch_one(const LevelGeom& g, int colour, const void* b, void* x, hipStream_t st) {
  constexpr int PPW = SmootherShape<D, K>::PPW, NT = SmootherShape<D, K>::NT;
  const int half = (int)(g.ncells / 2);
  int p[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) {
    p[a] = (colour >> a) & 1;
    cnt[a] = half - p[a];
  }
  for (int a = 0; a < D; ++a)
    if (cnt[a] <= 0) return hipSuccess;  // empty colour (coarsest level)
  const int groups0 = (cnt[0] + PPW - 1) / PPW;
  const long long blocks = (long long)groups0 * cnt[1] * (D == 3 ? cnt[2] : 1);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  // the kernel addresses one workgroup's block with 32-bit offsets
  constexpr long long n = 2 * K + 1;
  const long long span = (D == 3 ? (n - 1) * g.n1d * g.n1d : 0) + (n - 1) * g.n1d + 2 * K * PPW + 1;
  if (span >= (1LL << 31)) return hipErrorInvalidValue;
  // Abar_h = h^(d-2) Abar_1 ; A_j,h^{-1} = h^(2-d) A_j,1^{-1}
  const double h = g.h;
  const T res_scale = (T)(D == 3 ? h : 1.0);
  const T sol_scale = (T)(D == 3 ? 1.0 / h : 1.0);
  hipLaunchKernelGGL((colour_pass_kernel<D, K, T, ADD>), dim3((unsigned)blocks), dim3(NT), 0, st,
                     (const T*)b, (T*)x, g.n1d, p[0], p[1], p[2], cnt[0], cnt[1], groups0, res_scale, sol_scale);
  return hipGetLastError();
}

template <int D, int K>
static hipError_t dispatch_prec(const LevelGeom& g, int prec, bool add, int colour, const void* b, void* x,
                                hipStream_t st) {
  if (prec == 0)
    return add ? launch_one<D, K, double, true>(g, colour, b, x, st) : launch_one<D, K, double, false>(g, colour, b, x, st);
  return add ? launch_one<D, K, float, true>(g, colour, b, x, st) : launch_one<D, K, float, false>(g, colour, b, x, st);
}

template <int D>
static hipError_t dispatch_k(const LevelGeom& g, int prec, bool add, int colour, const void* b, void* x,
                             hipStream_t st) {
  switch (g.k) {
    case 1: return dispatch_prec<D, 1>(g, prec, add, colour, b, x, st);
    case 2: return dispatch_prec<D, 2>(g, prec, add, colour, b, x, st);
    case 3: return dispatch_prec<D, 3>(g, prec, add, colour, b, x, st);
    case 4: return dispatch_prec<D, 4>(g, prec, add, colour, b, x, st);
    case 5: return dispatch_prec<D, 5>(g, prec, add, colour, b, x, st);
    case 6: return dispatch_prec<D, 6>(g, prec, add, colour, b, x, st);
    case 7: return dispatch_prec<D, 7>(g, prec, add, colour, b, x, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_colour_pass(const LevelGeom& g, int prec, bool additive, int colour, const void* b, void* x,
                              hipStream_t st) {
  return g.dim == 2 ? dispatch_k<2>(g, prec, additive, colour, b, x, st)
                    : dispatch_k<3>(g, prec, additive, colour, b, x, st);
}

hipError_t init_smoother_tables() {
  static DevTables<double> h64[kMaxDegree + 1];
  static DevTables<float> h32[kMaxDegree + 1];
  for (int k = 1; k <= kMaxDegree; ++k) {
    fill_dev_tables(k, h64[k]);
    fill_dev_tables(k, h32[k]);
  }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tab64), h64, sizeof(h64));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tab32), h32, sizeof(h32));
}

}  // namespace vps
