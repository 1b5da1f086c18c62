// Matrix-free operator, residual, restriction and prolongation for gfx950.
//
// On a uniform Cartesian mesh the assembled operator is
//   A = sum_dir (x)_a (A1 if a == dir else M1)      (Sec. 2.3 eq:mf, eq:tensorproduct)
// with assembled 1D matrices A1 = sum_cells Ahat/h, M1 = sum_cells h Mhat, whose
// row of a node only depends on the node's position inside its cell (the
// "class" c = i mod k): 2k+1 band entries for a vertex, k+1 for a cell-interior
// node.  The kernels apply A by sum factorisation over node tiles:
//   stage x0: every thread reads one row of the input block (straight from
//             global memory into registers) and produces M1 x and A1 x along
//             x0 for the tile's outputs;
//   stage x1: one column per thread, out of LDS, U = M1 (M1 x), V = A1 (M1 x)
//             + M1 (A1 x) (3D) -- partial products reused as in the smoother;
//   stage x2: one column per thread, y = A1 U + M1 V, written to global.
// Each output node is owned by exactly one tile, so the result is
// deterministic and needs no atomics (the paper resolves cell overlaps with
// atomics; on a Cartesian mesh the node-tile form needs none).  Band classes
// are compile-time inside the unrolled tile loops, so structural zeros are
// skipped at compile time.
//
// Transfers use the same scheme with the 1D prolongation P1[i_f, J] =
// phi^coarse_J(x^fine_i) (Sec. 2.1: embedding by interpolation) and its
// transpose for restriction.
//
// All kernels here write interior nodes only; boundary entries of outputs are
// zeroed by zero_boundary_kernel where the caller needs it.
#include <mutex>
#include <string>

#include "device_common.hpp"
#include "patch_tables_gen.hpp"
#include "kernels.hpp"

namespace vps {

__device__ __forceinline__ bool is_bnd(long long i, long long n1d) { return i <= 0 || i >= n1d - 1; }

// Load n values of one row, positions g0 .. g0+n-1, as zero outside the interior (1 .. n1d-2).
// `interior` (wave-uniform) says the whole range is interior: then the loads are unconditional.
template <typename T, int N>
__device__ __forceinline__ void load_row(T (&in)[N], const T* __restrict__ row, long long g0, long long n1d,
                                         bool interior, bool row_ok) {
  if (interior) {
    const T* p = row + g0;
#pragma unroll
    for (int j = 0; j < N; ++j) in[j] = p[j];
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const long long g = g0 + j;
      const long long gc = g < 0 ? 0 : (g > n1d - 1 ? n1d - 1 : g);
      const T v = row[gc];
      in[j] = (g <= 0 || g >= n1d - 1) ? T(0) : v;
    }
  }
  if (!row_ok) {
#pragma unroll
    for (int j = 0; j < N; ++j) in[j] = T(0);
  }
}

// ----------------------------------------------------------------- operator

// Cells per tile along (x0, x1, x2).  2D: a task is one cell of one row (stage x0) or of one
// column (stage x1), so a tile of C0 x C1 cells has (K (C1 + 1) + 1) C0 and K C0 C1 tasks.  For
// degrees 2-7 C0 makes the x0 stage one round of the 256-thread workgroup (232-252 tasks); two
// rounds, with tiles of about 64 output columns, measured 20-28% slower at degrees 3-7 (FP64 apply,
// 2D levels of 4-13M nodes).  Degree 1 keeps 64-cell rows (narrower tiles measured slower).
template <int D, int K>
struct OpShape {
  static constexpr int C0 = D == 2 ? (K == 1 ? 64 : K == 2 ? 13 : K == 3 ? 9 : K <= 6 ? 8 : 7) : (16 / K > 1 ? 16 / K : 1);
  static constexpr int C1 = D == 2 ? (K == 1 ? 16 : K <= 3 ? 8 : K == 4 ? 6 : K == 5 ? 5 : 4)
                                   : (K == 1 ? 8 : K <= 4 ? 2 : 1);
  static constexpr int C2 = D == 3 ? C1 : 1;
  static constexpr int NT = D == 2 || K <= 4 ? 256 : 128;
};

template <int D, int K, typename T, bool RESID>
__global__ __launch_bounds__((OpShape<D, K>::NT)) void op_tile_kernel(const T* __restrict__ x, const T* __restrict__ b,
                                                                     T* __restrict__ y, long long n1d, int tiles0,
                                                                     int tiles1, T scale, double* __restrict__ pq_part) {
  using S = OpShape<D, K>;
  constexpr int NT = S::NT, W = 2 * K + 1;
  constexpr int TO0 = K * S::C0, TO1 = K * S::C1, TO2 = K * S::C2;
  constexpr int TI0 = TO0 + K + 1, TI1 = TO1 + K + 1, TI2 = D == 3 ? TO2 + K + 1 : 1;
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles0;
  const int ty = (blk / tiles0) % tiles1;
  const int tz = D == 3 ? blk / (tiles0 * tiles1) : 0;
  const long long o0 = (long long)tx * TO0, o1 = (long long)ty * TO1, o2 = (long long)tz * TO2;  // first output node
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x;

  __shared__ T PM[TI2 * TI1 * TO0];
  __shared__ T PA[TI2 * TI1 * TO0];
  // 2D FP64 x.y partials: x at the tile's output nodes, kept from stage x0
  constexpr bool XS = D == 2 && sizeof(T) == 8 && !RESID;
  __shared__ T XO[XS ? TO1 * TO0 : 1];
  const bool keep_x = XS && pq_part;

  // stage x0: rows (z, y) of the input block; 2D: cells of those rows (direct row loads: staging
  // the block in LDS first measured slower, it costs occupancy)
  const bool xin = o0 - K >= 1 && o0 - K + TI0 - 1 <= n1d - 2;
  if constexpr (D == 2) {
    for (int task = tid; task < TI1 * S::C0; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int yl = task / S::C0, cx = task - yl * S::C0;
      const long long gy = o1 - K + yl;
      const long long gyc = gy < 0 ? 0 : (gy > n1d - 1 ? n1d - 1 : gy);
      // nodes [vertex - K, vertex + K] around the cell's left vertex o0 + cx K
      T in[W];
      load_row<T, W>(in, x + gyc * n1d, o0 + cx * K - K, n1d, xin, !is_bnd(gy, n1d));
#pragma unroll
      for (int c = 0; c < K; ++c) {
        T sm = T(0), sa = T(0);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (c > 0 && t < K) continue;
          sm = fma_tab(CT::Mb[c * W + t], in[t], sm);
          sa = fma_tab(CT::Ab[c * W + t], in[t], sa);
        }
        PM[yl * TO0 + cx * K + c] = sm;
        PA[yl * TO0 + cx * K + c] = sa;
      }
      if (keep_x && yl >= K && yl < K + TO1) {
#pragma unroll
        for (int c = 0; c < K; ++c) XO[(yl - K) * TO0 + cx * K + c] = in[K + c];
      }
    }
  } else {
    for (int task = tid; task < TI2 * TI1; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int zl = task / TI1, yl = task - zl * TI1;
      const long long gz = o2 - K + zl, gy = o1 - K + yl;
      T in[TI0];
      const bool row_ok = !is_bnd(gy, n1d) && !is_bnd(gz, n1d);
      const long long gzc = gz < 0 ? 0 : (gz > n1d - 1 ? n1d - 1 : gz), gyc = gy < 0 ? 0 : (gy > n1d - 1 ? n1d - 1 : gy);
      load_row<T, TI0>(in, x + gzc * n1d2 + gyc * n1d, o0 - K, n1d, xin, row_ok);
#pragma unroll
      for (int xo = 0; xo < TO0; ++xo) {
        const int c = xo % K;
        T sm = T(0), sa = T(0);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (c > 0 && t < K) continue;
          sm = fma_tab(CT::Mb[c * W + t], in[xo - c + t], sm);
          sa = fma_tab(CT::Ab[c * W + t], in[xo - c + t], sa);
        }
        PM[(zl * TI1 + yl) * TO0 + xo] = sm;
        PA[(zl * TI1 + yl) * TO0 + xo] = sa;
      }
    }
  }
  __syncthreads();

  if constexpr (D == 2) {
    // stage x1: columns xo, outputs y = A1 (M1 x) + M1 (A1 x)
    // pq_part (FP64 only): as in the streaming form, the block's partial sum of x_i y_i, or of
    // (b - A x)_i^2 with the residual not stored
    double pq = 0.0;
    for (int task = tid; task < TO0 * S::C1; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int cy = task / TO0, xo = task - cy * TO0;
      // rows [vertex - K, vertex + K] around the cell's lower vertex o1 + cy K
      T pm[W], pa[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        pm[j] = PM[(cy * K + j) * TO0 + xo];
        pa[j] = PA[(cy * K + j) * TO0 + xo];
      }
      const long long gx = o0 + xo;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int yo = cy * K + c;
        T s = T(0);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (c > 0 && t < K) continue;
          s = fma_tab(CT::Ab[c * W + t], pm[t], s);
          s = fma_tab(CT::Mb[c * W + t], pa[t], s);
        }
        const long long gy = o1 + yo;
        if (!is_bnd(gx, n1d) && !is_bnd(gy, n1d)) {
          const long long g = gy * n1d + gx;
          const T v = RESID ? b[g] - scale * s : scale * s;
          if (sizeof(T) == 8 && RESID && pq_part) {
            pq = fma((double)v, (double)v, pq);
          } else {
            y[g] = v;
            if (keep_x) pq = fma((double)XO[yo * TO0 + xo], (double)v, pq);
          }
        }
      }
    }
    if constexpr (sizeof(T) == 8) {
      if (pq_part) {
        // fixed-order block reduction
        __shared__ double red[NT];
        red[tid] = pq;
        __syncthreads();
        for (int w = 1; w < NT; w *= 2) {
          if (tid % (2 * w) == 0 && tid + w < NT) red[tid] += red[tid + w];
          __syncthreads();
        }
        if (tid == 0) pq_part[blockIdx.x] = red[0];
      }
    }
  } else {
    __shared__ T U[TI2 * TO1 * TO0];
    __shared__ T V[TI2 * TO1 * TO0];
    // stage x1: columns (z, xo)
    for (int task = tid; task < TI2 * TO0; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int zl = task / TO0, xo = task - zl * TO0;
      T pm[TI1], pa[TI1];
#pragma unroll
      for (int j = 0; j < TI1; ++j) {
        pm[j] = PM[(zl * TI1 + j) * TO0 + xo];
        pa[j] = PA[(zl * TI1 + j) * TO0 + xo];
      }
#pragma unroll
      for (int yo = 0; yo < TO1; ++yo) {
        const int c = yo % K;
        T su = T(0), sv = T(0);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (c > 0 && t < K) continue;
          su = fma_tab(CT::Mb[c * W + t], pm[yo - c + t], su);
          sv = fma_tab(CT::Ab[c * W + t], pm[yo - c + t], sv);
          sv = fma_tab(CT::Mb[c * W + t], pa[yo - c + t], sv);
        }
        U[(zl * TO1 + yo) * TO0 + xo] = su;
        V[(zl * TO1 + yo) * TO0 + xo] = sv;
      }
    }
    __syncthreads();
    // stage x2: columns (yo, xo); y = A1 U + M1 V
    for (int task = tid; task < TO1 * TO0; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int yo = task / TO0, xo = task - yo * TO0;
      T u[TI2], v[TI2];
#pragma unroll
      for (int j = 0; j < TI2; ++j) {
        u[j] = U[(j * TO1 + yo) * TO0 + xo];
        v[j] = V[(j * TO1 + yo) * TO0 + xo];
      }
      const long long gx = o0 + xo, gy = o1 + yo;
      const bool col_ok = !is_bnd(gx, n1d) && !is_bnd(gy, n1d);
#pragma unroll
      for (int zo = 0; zo < TO2; ++zo) {
        const int c = zo % K;
        T s = T(0);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          if (c > 0 && t < K) continue;
          s = fma_tab(CT::Ab[c * W + t], u[zo - c + t], s);
          s = fma_tab(CT::Mb[c * W + t], v[zo - c + t], s);
        }
        const long long gz = o2 + zo;
        if (col_ok && !is_bnd(gz, n1d)) {
          const long long g = gz * n1d2 + gy * n1d + gx;
          y[g] = RESID ? b[g] - scale * s : scale * s;
        }
      }
    }
  }
}

// ------------------------------------------------- operator, 3D streaming form
//
// y = A2 (M1 M0 x) + M2 (A1 M0 x + M1 A0 x) with the assembled 1D matrices applied in cell
// form: along each axis a cell c contributes Ahat/Mhat (reference cell, compile-time indices,
// SGPR operands) to its K+1 nodes, a vertex sums the contributions of its two cells.  A
// workgroup owns a TX x TY column tile of the (x0, x1) plane and walks a chunk of cells along
// x2: every node plane is loaded once into LDS (with a K-node halo in x0 and x1 only), reduced
// in-plane (x0 then x1), and the x2 contraction runs in registers over the K+1 planes of the
// current cell, carrying the left-cell part of the next vertex.  The z halo is one cell per
// chunk instead of per tile, which removes most of the recomputation of a cubic tile.

template <int K>
struct OpStream {
  static constexpr int CX = K == 1 ? 16 : K == 2 ? 8 : K == 3 ? 5 : K == 4 ? 4 : K == 5 ? 3 : 2;
  static constexpr int TX = K * CX, TY = K * CX;        // outputs per plane tile
  static constexpr int NT = TX * TY;                    // one thread per output column
  static constexpr int IX = TX + K + 1, IY = TY + K + 1;  // input extents [o - K, o + T]
};

// pq_part != null: pq_part[block] = the block's partial sum in FP64 of x_i y_i (y = A x: the CG
// product p.Ap) or, for the residual, of r_i^2 with r = b - A x, which is then not stored (y may be
// null): the norm of the true residual.
template <int K, typename T, bool RESID>
__global__ __launch_bounds__((OpStream<K>::NT)) void op_stream_kernel(const T* __restrict__ x, const T* __restrict__ b,
                                                                     T* __restrict__ y, long long n1d, int tiles0,
                                                                     int tiles1, int cz, T scale,
                                                                     double* __restrict__ pq_part) {
  using S = OpStream<K>;
  constexpr int NT = S::NT, TX = S::TX, TY = S::TY, IX = S::IX, IY = S::IY, CX = S::CX, NP = K + 1;
  constexpr int PL = IY * IX;                  // values of one input plane tile
  constexpr int RB = (K * PL + NT - 1) / NT;   // prefetch registers per thread (one cell of planes)
  constexpr int XS = K * PL > 2 * K * TY * TX ? K * PL : 2 * K * TY * TX;
  // X (input planes) and, once X is consumed, Pm / Pq (in-plane results) share one buffer
  __shared__ T XP[XS];
  __shared__ T Rm[K * IY * TX];  // M0 x, [plane][r][c]
  __shared__ T Ra[K * IY * TX];  // A0 x
  T* X = XP;
  T* Pm = XP;                    // M1 M0 x, [plane][r][c]
  T* Pq = XP + K * TY * TX;      // A1 M0 x + M1 A0 x

  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles0;
  const int ty = (blk / tiles0) % tiles1;
  const int chunk = blk / (tiles0 * tiles1);
  const long long o0 = (long long)tx * TX, o1 = (long long)ty * TY;
  const long long ncz = (n1d - 1) / K;  // cells along x2
  const long long g0 = (long long)chunk * cz;
  const long long g1 = g0 + cz < ncz ? g0 + cz : ncz;
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x;
  const int px = tid % TX, py = tid / TX;
  const long long gx = o0 + px, gy = o1 + py;
  const bool col_out = !is_bnd(gx, n1d) && !is_bnd(gy, n1d) && gx < n1d && gy < n1d;

  // registers <- nb node planes zs .. zs+nb-1 of the tile (Dirichlet and outside nodes 0).
  // Element i = rr NT + tid of a fetch is node (plane i / PL, row, column) of the tile.  Its byte
  // offset from plane zs is the same in every fetch, so it is computed once, for the node clamped
  // into the grid: every fetch loads every element unconditionally (no branches) and a select
  // zeroes the elements that are not interior nodes.  Bit 31 of the offset marks a node outside
  // the interior in x0 or x1 (offsets stay below 2^31, checked by the launcher); the planes valid
  // in a fetch form the offset range [jlo, jhi) planes, known to the whole workgroup, which the
  // marked offsets never fall into.
  T pre[RB];
  unsigned poff[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int i = rr * NT + tid;
    const int j = i / PL, rem = i - j * PL;
    const int r = rem / IX, c = rem - r * IX;
    const long long sy = o1 - K + r, sx = o0 - K + c;
    const bool ok = i < K * PL && sy >= 1 && sy <= n1d - 2 && sx >= 1 && sx <= n1d - 2;
    const long long cy = sy < 0 ? 0 : sy > n1d - 1 ? n1d - 1 : sy;
    const long long cx = sx < 0 ? 0 : sx > n1d - 1 ? n1d - 1 : sx;
    const long long cj = j < K ? j : K - 1;
    poff[rr] = (unsigned)((cj * n1d2 + cy * n1d + cx) * (long long)sizeof(T)) | (ok ? 0u : 0x80000000u);
  }
  const unsigned plane_bytes = (unsigned)(n1d2 * (long long)sizeof(T));
  // fetches only ever cover planes 0 .. n1d-1: zs >= 0 and zs + K - 1 <= n1d - 1
  auto fetch = [&](long long zs, int nb) {
    const unsigned jlo = zs < 1 ? (unsigned)(1 - zs) : 0u;
    const unsigned jhi = (unsigned)(zs + nb <= n1d - 1 ? nb : n1d - 1 - zs);
    const unsigned lo = jlo * plane_bytes, span = jhi * plane_bytes - lo;
    const T* plane = x + zs * n1d2;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const T v = ld_lane(plane, poff[rr] & 0x7fffffffu);
      pre[rr] = poff[rr] - lo < span ? v : T(0);
    }
  };
  auto stage = [&](int nb) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int i = rr * NT + tid;
      if (i < nb * PL) X[i] = pre[rr];
    }
  };
  // X (nb planes) -> Pm, Pq (nb planes); ends after a barrier, results readable by every thread
  auto reduce = [&](int nb) {
    __syncthreads();
    for (int task = tid; task < nb * IY * CX; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int j = task / (IY * CX), rem = task - j * (IY * CX);
      const int r = rem / CX, cx = rem - r * CX;
      T in[2 * K + 1];
#pragma unroll
      for (int t = 0; t <= 2 * K; ++t) in[t] = X[j * PL + r * IX + cx * K + t];
#pragma unroll
      for (int li = 0; li < K; ++li) {
        T sm = T(0), sa = T(0);
        if (li == 0) {
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            sm = fma_tab(CT::Mh[K * NP + q], in[q], sm);
            sa = fma_tab(CT::Ah[K * NP + q], in[q], sa);
          }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          sm = fma_tab(CT::Mh[li * NP + q], in[K + q], sm);
          sa = fma_tab(CT::Ah[li * NP + q], in[K + q], sa);
        }
        Rm[(j * IY + r) * TX + cx * K + li] = sm;
        Ra[(j * IY + r) * TX + cx * K + li] = sa;
      }
    }
    __syncthreads();
    for (int task = tid; task < nb * TX * CX; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int j = task / (TX * CX), rem = task - j * (TX * CX);
      const int cy = rem / TX, c = rem - cy * TX;
      T im[2 * K + 1], ia[2 * K + 1];
#pragma unroll
      for (int t = 0; t <= 2 * K; ++t) {
        im[t] = Rm[(j * IY + cy * K + t) * TX + c];
        ia[t] = Ra[(j * IY + cy * K + t) * TX + c];
      }
#pragma unroll
      for (int li = 0; li < K; ++li) {
        T su = T(0), sv = T(0);
        if (li == 0) {
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            su = fma_tab(CT::Mh[K * NP + q], im[q], su);
            sv = fma_tab(CT::Ah[K * NP + q], im[q], sv);
            sv = fma_tab(CT::Mh[K * NP + q], ia[q], sv);
          }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          su = fma_tab(CT::Mh[li * NP + q], im[K + q], su);
          sv = fma_tab(CT::Ah[li * NP + q], im[K + q], sv);
          sv = fma_tab(CT::Mh[li * NP + q], ia[K + q], sv);
        }
        Pm[(j * TY + cy * K + li) * TX + c] = su;
        Pq[(j * TY + cy * K + li) * TX + c] = sv;
      }
    }
    __syncthreads();
  };

  // x2 in cell form: cell g spans node planes gK .. gK+K; zm/zq[0] is its left plane
  T zm[NP], zq[NP];
  T carry = T(0);
  double pq = 0.0;
  zm[0] = zq[0] = T(0);
  if (g0 > 0) {
    fetch((g0 - 1) * K, 1);
    stage(1);
    fetch((g0 - 1) * K + 1, K);
    reduce(1);
    zm[0] = Pm[tid];
    zq[0] = Pq[tid];
    __syncthreads();
    stage(K);
    fetch(g0 * K + 1, K);
    reduce(K);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      zm[1 + j] = Pm[j * TY * TX + tid];
      zq[1 + j] = Pq[j * TY * TX + tid];
    }
    __syncthreads();
    using CT = gen::CellTables<T, K>;
#pragma unroll
    for (int j = 0; j < NP; ++j) carry = fma_tab(CT::Ah[K * NP + j], zm[j], fma_tab(CT::Mh[K * NP + j], zq[j], carry));
    zm[0] = zm[K];
    zq[0] = zq[K];
  } else {
    fetch(1, K);
  }
  for (long long g = g0; g < g1; ++g) {
    stage(K);
    if (g + 1 < g1) fetch((g + 1) * K + 1, K);
    reduce(K);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      zm[1 + j] = Pm[j * TY * TX + tid];
      zq[1 + j] = Pq[j * TY * TX + tid];
    }
    __syncthreads();
    using CT = gen::CellTables<T, K>;
#pragma unroll
    for (int li = 0; li < K; ++li) {
      T s = li == 0 ? carry : T(0);
#pragma unroll
      for (int j = 0; j < NP; ++j) s = fma_tab(CT::Ah[li * NP + j], zm[j], fma_tab(CT::Mh[li * NP + j], zq[j], s));
      const long long zg = g * K + li;
      if (col_out && zg >= 1) {
        const long long gi = zg * n1d2 + gy * n1d + gx;
        const T v = RESID ? b[gi] - scale * s : scale * s;
        if (RESID && sizeof(T) == 8 && pq_part) {
          pq = fma((double)v, (double)v, pq);
        } else {
          y[gi] = v;
          if (!RESID && pq_part) pq = fma((double)x[gi], (double)v, pq);
        }
      }
    }
    carry = T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) carry = fma_tab(CT::Ah[K * NP + j], zm[j], fma_tab(CT::Mh[K * NP + j], zq[j], carry));
    zm[0] = zm[K];
    zq[0] = zq[K];
  }
  // (the FP32 residual never takes partial sums: no reduction buffer for it)
  if (pq_part && (!RESID || sizeof(T) == 8)) {
    // fixed-order block reduction (the LDS buffers are free after the last barrier of the loop)
    __shared__ double red[NT];
    red[tid] = pq;
    __syncthreads();
    for (int w = 1; w < NT; w *= 2) {
      if (tid % (2 * w) == 0 && tid + w < NT) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) pq_part[blockIdx.x] = red[0];
  }
}

// ----------------------------------------------------------- prolongation

// Coarse cells per tile and threads: 3D cubic tiles (degree 1 only; the other degrees take the
// tiles of prolong3_kernel below) span 2kC ~ 16 fine nodes per axis, so the last stage (one thread
// per fine column) fills a 256-thread workgroup.  2D: a task is one coarse cell of one row (stage
// x0) or of one fine column (stage x1); a tile of C0 x C1 coarse cells (about 64 fine columns by
// 8k fine rows) makes both stages one round of the workgroup: (k C1 + 1) C0 and 2k C0 C1 tasks,
// at most 256.  Square tiles took up to 8 rounds at degrees 1-4: 2D V-cycles 6% (degrees 1, 2),
// 2-3% (3, 4) slower, equal at 5-7.
template <int D, int K>
struct ProShape {
  static constexpr int C = D == 2 ? 4 : (K == 1 ? 8 : K == 2 ? 4 : K <= 4 ? 2 : 1);  // 3D: cubic tiles
  static constexpr int C0 = D == 2 ? (K == 1 ? 32 : K == 2 ? 16 : K == 3 ? 10 : K == 4 ? 8 : K == 5 ? 6 : K == 6 ? 5 : 4) : C;
  static constexpr int C1 = D == 2 ? 4 : C;
  static constexpr int NT = D == 2 || K <= 4 ? 256 : 128;
};

// x_fine += P e_coarse.  Tile: coarse cells [C t, C (t+1)) per axis, fine outputs
// [2kC t, 2kC (t+1)), coarse inputs [kC t, kC (t+1)].
template <int D, int K, typename T>
__global__ __launch_bounds__((ProShape<D, K>::NT)) void prolong_tile_kernel(const T* __restrict__ e, T* __restrict__ xf,
                                                                          long long n1dc, long long n1df, int tiles0,
                                                                          int tiles1) {
  constexpr int C = ProShape<D, K>::C, C0 = ProShape<D, K>::C0, C1 = ProShape<D, K>::C1, NT = ProShape<D, K>::NT;
  constexpr int TI = K * C + 1, TO = 2 * K * C, TIz = D == 3 ? TI : 1;
  constexpr int TI1 = K * C1 + 1, TO0 = 2 * K * C0;  // 2D tile: coarse rows, fine columns
  constexpr int NP = K + 1;
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles0, ty = (blk / tiles0) % tiles1, tz = D == 3 ? blk / (tiles0 * tiles1) : 0;
  const long long c0 = (long long)tx * K * C0, c1 = (long long)ty * K * C1, c2 = (long long)tz * K * C;
  const long long f0 = 2 * c0, f1 = 2 * c1, f2 = 2 * c2;
  const int tid = threadIdx.x;
  const long long nc2 = n1dc * n1dc, nf2 = n1df * n1df;
  __shared__ T T1[D == 2 ? TI1 * TO0 : TIz * TI * TO];
  if constexpr (D == 2) {
    // stage x0: coarse cells cc of coarse rows yl
    for (int task = tid; task < TI1 * C0; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int yl = task / C0, cc = task - yl * C0;
      const long long gy = c1 + yl;
      const bool ok = gy < n1dc && !is_bnd(gy, n1dc);
      const long long row = min(gy, n1dc - 1) * n1dc;
      T in[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) in[a] = e[row + min(c0 + K * cc + a, n1dc - 1)];
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        const long long gx = c0 + K * cc + a;
        if (!(ok && gx < n1dc && !is_bnd(gx, n1dc))) in[a] = T(0);
      }
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          if (q == 0 && a > 0) continue;
          s = fma_tab(CT::P[q * NP + a], in[a], s);
        }
        T1[yl * TO0 + 2 * K * cc + q] = s;
      }
    }
    __syncthreads();
    // stage x1: coarse cells cc of fine columns xo; the thread's outputs are its own, every old value
    // is loaded before the first store
    for (int task = tid; task < TO0 * C1; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int cc = task / TO0, xo = task - cc * TO0;
      T in[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) in[a] = T1[(K * cc + a) * TO0 + xo];
      const long long gx = f0 + xo;
      T old[2 * K];
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) {
        const long long gy = f1 + 2 * K * cc + q;
        old[q] = gx < n1df && gy < n1df && !is_bnd(gx, n1df) && !is_bnd(gy, n1df) ? xf[gy * n1df + gx] : T(0);
      }
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          if (q == 0 && a > 0) continue;
          s = fma_tab(CT::P[q * NP + a], in[a], s);
        }
        const long long gy = f1 + 2 * K * cc + q;
        if (gx < n1df && gy < n1df && !is_bnd(gx, n1df) && !is_bnd(gy, n1df)) xf[gy * n1df + gx] = old[q] + s;
      }
    }
  } else {
    // stage x0: coarse rows
    for (int task = tid; task < TIz * TI; task += NT) {
      using CT = gen::CellTables<T, K>;
      const int zl = task / TI, yl = task - zl * TI;
      const long long gz = c2 + zl, gy = c1 + yl;
      const bool ok = gy < n1dc && !is_bnd(gy, n1dc) && gz < n1dc && !is_bnd(gz, n1dc);
      // every load of the row first, at indices clamped into the grid; out-of-range values taken as 0
      const long long row = min(gz, n1dc - 1) * nc2 + min(gy, n1dc - 1) * n1dc;
      T in[TI];
#pragma unroll
      for (int j = 0; j < TI; ++j) in[j] = e[row + min(c0 + j, n1dc - 1)];
#pragma unroll
      for (int j = 0; j < TI; ++j) {
        const long long gx = c0 + j;
        if (!(ok && gx < n1dc && !is_bnd(gx, n1dc))) in[j] = T(0);
      }
#pragma unroll
      for (int xo = 0; xo < TO; ++xo) {
        const int cc = xo / (2 * K), q = xo % (2 * K);
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          if (q == 0 && a > 0) continue;
          s = fma_tab(CT::P[q * NP + a], in[K * cc + a], s);
        }
        T1[(zl * TI + yl) * TO + xo] = s;
      }
    }
    __syncthreads();
    {
      __shared__ T T2[TI * TO * TO];
      for (int task = tid; task < TI * TO; task += NT) {
        using CT = gen::CellTables<T, K>;
        const int zl = task / TO, xo = task - zl * TO;
        T in[TI];
#pragma unroll
        for (int j = 0; j < TI; ++j) in[j] = T1[(zl * TI + j) * TO + xo];
#pragma unroll
        for (int yo = 0; yo < TO; ++yo) {
          const int cc = yo / (2 * K), q = yo % (2 * K);
          T s = T(0);
#pragma unroll
          for (int a = 0; a < NP; ++a) {
            if (q == 0 && a > 0) continue;
            s = fma_tab(CT::P[q * NP + a], in[K * cc + a], s);
          }
          T2[(zl * TO + yo) * TO + xo] = s;
        }
      }
      __syncthreads();
      for (int task = tid; task < TO * TO; task += NT) {
        using CT = gen::CellTables<T, K>;
        const int yo = task / TO, xo = task - yo * TO;
        T in[TI];
#pragma unroll
        for (int j = 0; j < TI; ++j) in[j] = T2[(j * TO + yo) * TO + xo];
        const long long gx = f0 + xo, gy = f1 + yo;
        const bool ok = gx < n1df && gy < n1df && !is_bnd(gx, n1df) && !is_bnd(gy, n1df);
        // the thread's outputs are its own (tiles do not overlap): every old value is loaded before
        // the first store, so the loads are in flight together instead of one after each store
        T old[TO];
#pragma unroll
        for (int zo = 0; zo < TO; ++zo) {
          const long long gz = f2 + zo;
          old[zo] = ok && gz < n1df && !is_bnd(gz, n1df) ? xf[gz * nf2 + gy * n1df + gx] : T(0);
        }
#pragma unroll
        for (int zo = 0; zo < TO; ++zo) {
          const int cc = zo / (2 * K), q = zo % (2 * K);
          T s = T(0);
#pragma unroll
          for (int a = 0; a < NP; ++a) {
            if (q == 0 && a > 0) continue;
            s = fma_tab(CT::P[q * NP + a], in[K * cc + a], s);
          }
          const long long gz = f2 + zo;
          if (ok && gz < n1df && !is_bnd(gz, n1df)) xf[gz * nf2 + gy * n1df + gx] = old[zo] + s;
        }
      }
    }
  }
}

// 3D prolongation, tiles of C0 x C1 x C2 coarse cells: about 32 fine nodes along x0, 16 along x1
// and 8 along x2, so that the last stage reads and writes whole 128-byte row segments of x_fine.
// Every stage takes one coarse cell per task (its K+1 inputs, 2K outputs): one cell of a coarse
// row (x0), of a fine column along x1 (x1) and along x2 (x2).  Same arithmetic per output as the
// per-row form, in the same order.  Used for degrees >= 2 (3D Q4 64^3 solve -0.4%, degrees 2, 3
// and 7 equal); degree 1 measured slower (V-cycle +1.4% at 256^3 cells) and keeps the cubic tiles.
template <int K>
constexpr bool kPro3Tiles = K >= 2;
template <int K>
struct Pro3 {
  static constexpr int C0 = K == 1 ? 16 : K == 2 ? 8 : K == 3 ? 5 : K == 4 ? 4 : K <= 6 ? 3 : 2;
  static constexpr int C1 = K == 1 ? 8 : K == 2 ? 4 : K == 3 ? 3 : K <= 5 ? 2 : 1;
  static constexpr int C2 = K == 1 ? 4 : K == 2 ? 2 : 1;
  static constexpr int NT = 256;
};

template <int K, typename T>
__global__ __launch_bounds__(256) void prolong3_kernel(const T* __restrict__ e, T* __restrict__ xf, long long n1dc,
                                                       long long n1df, int tiles0, int tiles1) {
  using S = Pro3<K>;
  constexpr int NT = S::NT, NP = K + 1, R = 2 * K;
  constexpr int TO0 = R * S::C0, TO1 = R * S::C1, TO2 = R * S::C2;
  constexpr int TI1 = K * S::C1 + 1, TI2 = K * S::C2 + 1;
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles0, ty = (blk / tiles0) % tiles1, tz = blk / (tiles0 * tiles1);
  const long long c0 = (long long)tx * K * S::C0, c1 = (long long)ty * K * S::C1, c2 = (long long)tz * K * S::C2;
  const long long f0 = 2 * c0, f1 = 2 * c1, f2 = 2 * c2;
  const int tid = threadIdx.x;
  const long long nc2 = n1dc * n1dc, nf2 = n1df * n1df;
  __shared__ T T1[TI2 * TI1 * TO0];  // along x0: [coarse z][coarse y][fine x]
  __shared__ T T2[TI2 * TO1 * TO0];  // along x1: [coarse z][fine y][fine x]
  using CT = gen::CellTables<T, K>;
  for (int task = tid; task < TI2 * TI1 * S::C0; task += NT) {
    const int row = task / S::C0, cc = task - row * S::C0;
    const int zl = row / TI1, yl = row - zl * TI1;
    const long long gz = c2 + zl, gy = c1 + yl;
    const bool ok = gy < n1dc && !is_bnd(gy, n1dc) && gz < n1dc && !is_bnd(gz, n1dc);
    // every load first, at indices clamped into the grid; out-of-range values taken as 0
    const long long base = min(gz, n1dc - 1) * nc2 + min(gy, n1dc - 1) * n1dc;
    T in[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) in[a] = e[base + min(c0 + K * cc + a, n1dc - 1)];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const long long gx = c0 + K * cc + a;
      if (!(ok && gx < n1dc && !is_bnd(gx, n1dc))) in[a] = T(0);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        if (q == 0 && a > 0) continue;
        s = fma_tab(CT::P[q * NP + a], in[a], s);
      }
      T1[row * TO0 + R * cc + q] = s;
    }
  }
  __syncthreads();
  for (int task = tid; task < TI2 * S::C1 * TO0; task += NT) {
    const int col = task / TO0, xo = task - col * TO0;
    const int zl = col / S::C1, cc = col - zl * S::C1;
    T in[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) in[a] = T1[(zl * TI1 + K * cc + a) * TO0 + xo];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        if (q == 0 && a > 0) continue;
        s = fma_tab(CT::P[q * NP + a], in[a], s);
      }
      T2[(zl * TO1 + R * cc + q) * TO0 + xo] = s;
    }
  }
  __syncthreads();
  for (int task = tid; task < S::C2 * TO1 * TO0; task += NT) {
    const int col = task / TO0, xo = task - col * TO0;
    const int cc = col / TO1, yo = col - cc * TO1;
    T in[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) in[a] = T2[((K * cc + a) * TO1 + yo) * TO0 + xo];
    const long long gx = f0 + xo, gy = f1 + yo;
    const bool ok = gx < n1df && gy < n1df && !is_bnd(gx, n1df) && !is_bnd(gy, n1df);
    // the thread's outputs are its own: every old value is loaded before the first store
    T old[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const long long gz = f2 + R * cc + q;
      old[q] = ok && gz < n1df && !is_bnd(gz, n1df) ? xf[gz * nf2 + gy * n1df + gx] : T(0);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        if (q == 0 && a > 0) continue;
        s = fma_tab(CT::P[q * NP + a], in[a], s);
      }
      const long long gz = f2 + R * cc + q;
      if (ok && gz < n1df && !is_bnd(gz, n1df)) xf[gz * nf2 + gy * n1df + gx] = old[q] + s;
    }
  }
  static_assert(TO2 == R * S::C2, "tile extent along x2");
}

// ------------------------------------------------- restriction, 3D in two kernels
//
// rc = (P1 x P1 x P1)^T rf in cell form: along each axis the fine nodes are split into
// half-open runs 2KC .. 2KC + 2K - 1, one per coarse cell C, and each run maps to the K+1
// coarse nodes of its cell with P[q][a] = phi_a(fine position q); a coarse vertex sums the
// parts of its two cells (the fine node on the vertex lies in one run only, so every entry of
// P1 is used once).  Fine boundary nodes count as 0; coarse boundary nodes are written 0.
//  * restrict_plane_kernel: one workgroup per (GP fine planes, TX x TX coarse-column tile)
//    reduces the planes along x0 and x1 (LDS) into T[zf][J1][J0] (nc x nc per fine plane);
//  * restrict_z_kernel: one thread per (coarse column, two coarse cells along x2) combines T along x2.
// Every launch is fully parallel (no chain of dependent planes inside a workgroup), the fine
// vector is read once and the intermediate is a quarter of it.  Each thread issues all of its
// global loads before it uses any of them, so a workgroup waits for memory once, not once per
// element.

#ifndef VPS_RES_GP
#define VPS_RES_GP 2
#endif
template <int K, typename T>
struct ResPlane {
  static constexpr int CX = K == 1 ? 16 : K == 2 ? 8 : K == 3 ? 5 : K == 4 ? 4 : K == 5 ? 3 : 2;
  static constexpr int TX = K * CX;            // coarse columns per tile row
  static constexpr int NT = 256;
  static constexpr int IX = 2 * TX + 2 * K;    // fine extent [2o - 2K, 2o + 2TX - 1]
  static constexpr int GP = sizeof(T) == 4 ? VPS_RES_GP : (VPS_RES_GP + 1) / 2;  // fine planes per workgroup
  static constexpr int LPT = (IX * IX + NT - 1) / NT;       // loads per thread and plane
  // LDS row strides: odd for the fine tile, 2 mod 4 for the x0-reduced tile, so that the lanes of
  // a half-wave (consecutive rows) read different banks
  static constexpr int XS = IX | 1;
  static constexpr int RS = TX + (6 - TX % 4) % 4;
};

// in[t] = fine nodes 2K(C-1) + t, t < 4K (the runs of cells C-1 and C): coarse node a of cell C
template <int K, typename T>
__device__ __forceinline__ T restrict_run(const T* in, int a) {
  using CT = gen::CellTables<T, K>;
  constexpr int NP = K + 1, RUN = 2 * K;
  T s = T(0);
  if (a == 0) {
#pragma unroll
    for (int q = 0; q < RUN; ++q) s = fma(CT::P[q * NP + K], in[q], s);
  }
  // plain multiply-adds here: skipping the few zero entries of P breaks up the paired LDS reads of
  // `in` and made the kernel slower
#pragma unroll
  for (int q = 0; q < RUN; ++q) s = fma(CT::P[q * NP + a], in[RUN + q], s);
  return s;
}

template <int K, typename T>
__global__ __launch_bounds__(256) void restrict_plane_kernel(const T* __restrict__ rf, T* __restrict__ tz,
                                                            long long nf, long long nc, int tiles) {
  using S = ResPlane<K, T>;
  constexpr int NT = S::NT, TX = S::TX, IX = S::IX, CX = S::CX, RUN = 2 * K, GP = S::GP, LPT = S::LPT;
  constexpr int XS = S::XS, RS = S::RS;
  __shared__ T X[GP * IX * XS];
  __shared__ T Rx[GP * IX * RS];
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles, ty = blk / tiles;
  const int z0 = 1 + GP * (int)blockIdx.y;  // first interior fine plane of the group
  const int np = min(GP, (int)nf - 1 - z0);  // planes z0 .. z0 + np - 1 (<= nf - 2)
  const long long o0 = (long long)tx * TX, o1 = (long long)ty * TX;
  const int tid = threadIdx.x;
  // 32-bit offsets from the group's first plane (the launcher checks GP nf^2 words fit)
  const int nfi = (int)nf, fy0 = (int)(2 * o1) - 2 * K, fx0 = (int)(2 * o0) - 2 * K;
  const T* fz = rf + (long long)z0 * nf * nf;
  T v[GP][LPT];
#pragma unroll
  for (int j = 0; j < GP; ++j) {
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      const int i = tid + l * NT;
      const int r = i / IX, c = i - r * IX;
      const int fy = fy0 + r, fx = fx0 + c;
      const bool ok = j < np && i < IX * IX && fy >= 1 && fy <= nfi - 2 && fx >= 1 && fx <= nfi - 2;
      v[j][l] = ok ? ld_lane(fz, (unsigned)((j * nfi + fy) * nfi + fx) * (unsigned)sizeof(T)) : T(0);
    }
  }
#pragma unroll
  for (int j = 0; j < GP; ++j) {
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      const int i = tid + l * NT;
      const int r = i / IX, c = i - r * IX;
      if (i < IX * IX) X[(j * IX + r) * XS + c] = v[j][l];
    }
  }
  __syncthreads();
  for (int task = tid; task < GP * IX * CX; task += NT) {
    const int j = task / (IX * CX), e = task - j * (IX * CX);
    const int r = e / CX, cx = e - r * CX;
    T in[2 * RUN];
#pragma unroll
    for (int t = 0; t < 2 * RUN; ++t) in[t] = X[(j * IX + r) * XS + RUN * cx + t];
#pragma unroll
    for (int a = 0; a < K; ++a) Rx[(j * IX + r) * RS + cx * K + a] = restrict_run<K, T>(in, a);
  }
  __syncthreads();
  for (int task = tid; task < GP * TX * CX; task += NT) {
    const int j = task / (TX * CX), e = task - j * (TX * CX);
    if (j >= np) break;
    const int cy = e / TX, c = e - cy * TX;
    T in[2 * RUN];
#pragma unroll
    for (int t = 0; t < 2 * RUN; ++t) in[t] = Rx[(j * IX + RUN * cy + t) * RS + c];
    T* out = tz + (long long)(z0 + j) * nc * nc;
    const long long gx = o0 + c;
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const long long gy = o1 + cy * K + a;
      if (gx < nc && gy < nc) out[gy * nc + gx] = restrict_run<K, T>(in, a);
    }
  }
}

// ------------------------------------------------- restriction, 2D in one kernel
//
// The in-plane part of the 3D scheme on the whole 2D grid: a workgroup owns a TX x TX coarse tile,
// loads the fine nodes [2o - 2K, 2o + 2TX - 1] of both axes into LDS (fine boundary nodes as 0),
// reduces along x0 (cell runs, restrict_run) and then along x1, and writes its coarse nodes, 0 on
// the coarse boundary.  The tiles cover every coarse node; a non-null xz (the coarse iterate) is
// zeroed on the same nodes.
// Coarse cells per tile side, chosen so that the x0 stage (IX CX tasks: 220, 224, 252, 240, 200,
// 240, 168 for degrees 1-7) is one round of the workgroup.  Tiles of about 28 coarse nodes per
// side took up to 6 rounds: 2D V-cycles 1-5% slower at degrees 1-4 and 7, equal at 5.
template <int K, typename T>
struct Res2D {
  static constexpr int CX = K == 1 ? 10 : K == 2 ? 7 : K == 3 ? 6 : K == 4 ? 5 : K <= 6 ? 4 : 3;
  static constexpr int TX = K * CX;          // coarse nodes per tile side
  static constexpr int NT = 256;
  static constexpr int IX = 2 * TX + 2 * K;  // fine extent per side
  static constexpr int LPT = (IX * IX + NT - 1) / NT;
  static constexpr int XS = IX | 1;                      // odd row stride of the fine tile
  static constexpr int RS = TX + (6 - TX % 4) % 4;       // 2 mod 4 row stride of the x0-reduced tile
};

template <int K, typename T>
__global__ __launch_bounds__(256) void restrict_tile2d_kernel(const T* __restrict__ rf, T* __restrict__ rc,
                                                             T* __restrict__ xz, long long nf, long long nc,
                                                             int tiles) {
  using S = Res2D<K, T>;
  constexpr int NT = S::NT, TX = S::TX, IX = S::IX, CX = S::CX, RUN = 2 * K, LPT = S::LPT, XS = S::XS, RS = S::RS;
  __shared__ T X[IX * XS];
  __shared__ T Rx[IX * RS];
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = blk % tiles, ty = blk / tiles;
  const long long o0 = (long long)tx * TX, o1 = (long long)ty * TX;
  const long long fy0 = 2 * o1 - 2 * K, fx0 = 2 * o0 - 2 * K;
  const int tid = threadIdx.x;
  T v[LPT];
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    const int i = tid + l * NT;
    const int r = i / IX, c = i - r * IX;
    const long long fy = fy0 + r, fx = fx0 + c;
    const bool ok = i < IX * IX && fy >= 1 && fy <= nf - 2 && fx >= 1 && fx <= nf - 2;
    v[l] = ok ? rf[fy * nf + fx] : T(0);
  }
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    const int i = tid + l * NT;
    const int r = i / IX, c = i - r * IX;
    if (i < IX * IX) X[r * XS + c] = v[l];
  }
  __syncthreads();
  for (int task = tid; task < IX * CX; task += NT) {
    const int r = task / CX, cx = task - r * CX;
    T in[2 * RUN];
#pragma unroll
    for (int t = 0; t < 2 * RUN; ++t) in[t] = X[r * XS + RUN * cx + t];
#pragma unroll
    for (int a = 0; a < K; ++a) Rx[r * RS + cx * K + a] = restrict_run<K, T>(in, a);
  }
  __syncthreads();
  for (int task = tid; task < TX * CX; task += NT) {
    const int cy = task / TX, c = task - cy * TX;
    T in[2 * RUN];
#pragma unroll
    for (int t = 0; t < 2 * RUN; ++t) in[t] = Rx[(RUN * cy + t) * RS + c];
    const long long gx = o0 + c;
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const long long gy = o1 + cy * K + a;
      if (gx < nc && gy < nc) {
        const bool bnd = gx == 0 || gy == 0 || gx == nc - 1 || gy == nc - 1;
        rc[gy * nc + gx] = bnd ? T(0) : restrict_run<K, T>(in, a);
        if (xz) xz[gy * nc + gx] = T(0);
      }
    }
  }
}

// Workgroup = 64 x 4 coarse columns (x0 fastest); blockIdx.z = a pair of coarse cells along x2.  A
// thread loads the fine planes of the run before its first cell and of its cells' own runs (each
// run once), then for each cell C adds P[q][a] times each plane to the cell's coarse nodes.  Sums
// run in the same order as the node-by-node definition (previous run, then own run).
#ifndef VPS_RES_CPT
#define VPS_RES_CPT 2
#endif
constexpr int kResCellsPerThread = VPS_RES_CPT;
template <int K, typename T>
__global__ __launch_bounds__(256) void restrict_z_kernel(const T* __restrict__ tz, T* __restrict__ rc, int nf, int nc,
                                                        T* __restrict__ xz) {
  constexpr int NP = K + 1, RUN = 2 * K, CPT = kResCellsPerThread;
  using CT = gen::CellTables<T, K>;
  const int gx = blockIdx.x * 64 + threadIdx.x, gy = blockIdx.y * 4 + threadIdx.y;
  if (gx >= nc || gy >= nc) return;
  const int ncc = (nc - 1) / K;  // coarse cells along x2
  const int C0 = CPT * blockIdx.z;
  const long long nc2 = (long long)nc * nc;
  const unsigned off = (unsigned)(gy * nc + gx) * (unsigned)sizeof(T);  // within a plane
  const bool col = gx > 0 && gx < nc - 1 && gy > 0 && gy < nc - 1;     // else a boundary column: 0
  // run[j] = fine planes of cell C0 - 1 + j; planes outside [1, nf - 2] take no part (their loads
  // read a clamped, valid plane)
  T run[CPT + 1][RUN];
#pragma unroll
  for (int j = 0; j <= CPT; ++j) {
#pragma unroll
    for (int q = 0; q < RUN; ++q) {
      const int zf = min(max(RUN * (C0 - 1 + j) + q, 1), nf - 2);
      run[j][q] = ld_lane(tz + zf * nc2, off);
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int C = C0 + c;
    if (C >= ncc) break;
    T carry = T(0);  // the previous cell's contribution to this cell's first node
    if (C > 0) {
#pragma unroll
      for (int q = 0; q < RUN; ++q)
        if (RUN * (C - 1) + q >= 1) carry = fma(CT::P[q * NP + K], run[c][q], carry);
    }
    T s[NP];
    s[0] = carry;
#pragma unroll
    for (int a = 1; a < NP; ++a) s[a] = T(0);
#pragma unroll
    for (int q = 0; q < RUN; ++q) {
      const int zf = RUN * C + q;
      if (zf >= 1 && zf <= nf - 2) {
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          if (q == 0 && a > 0) continue;  // the run's first fine node is the coarse vertex itself
          s[a] = fma(CT::P[q * NP + a], run[c + 1][q], s[a]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const int zc = K * C + a;
      st_lane(rc + zc * nc2, off, col && zc > 0 ? s[a] : T(0));
      if (xz) st_lane(xz + zc * nc2, off, T(0));
    }
    if (C == ncc - 1) {
      st_lane(rc + (nc - 1) * nc2, off, T(0));  // the last coarse plane is a boundary plane
      if (xz) st_lane(xz + (nc - 1) * nc2, off, T(0));
    }
  }
}

// ------------------------------------------------------- boundary and rhs

// Zero every boundary node: thread per node of the d-1 dimensional faces.
template <typename T>
__global__ void zero_boundary_kernel(T* __restrict__ y, int dim, long long n1d) {
  const long long faces = dim == 2 ? n1d : n1d * n1d;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= faces) return;
  const long long n2 = n1d * n1d;
  for (int a = 0; a < dim; ++a) {
    // t enumerates the other axes; the boundary planes are index 0 and n1d-1 along axis a
    long long u = dim == 2 ? t : t % n1d, v = dim == 2 ? 0 : t / n1d;
    for (int side = 0; side < 2; ++side) {
      const long long fixed = side ? n1d - 1 : 0;
      long long idx;
      if (dim == 2)
        idx = a == 0 ? u * n1d + fixed : fixed * n1d + u;
      else
        idx = a == 0 ? (v * n1d + u) * n1d + fixed : a == 1 ? (v * n1d + fixed) * n1d + u : (fixed * n1d + v) * n1d + u;
      y[idx] = T(0);
    }
    (void)n2;
  }
}

// b[node] = sum_m coef[m] prod_a G[(m*dim + a)*n1d + i_a], interior nodes; boundary 0.
template <typename T>
__global__ void rhs_separable_kernel(T* __restrict__ b, const double* __restrict__ G, const double* __restrict__ coef,
                                     int nterms, int dim, long long n1d, long long ntot) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntot) return;
  const long long i0 = idx % n1d, r = idx / n1d;
  const long long i1 = r % n1d, i2 = dim == 3 ? r / n1d : 0;
  if (is_bnd(i0, n1d) || is_bnd(i1, n1d) || (dim == 3 && is_bnd(i2, n1d))) {
    b[idx] = T(0);
    return;
  }
  double s = 0.0;
  for (int m = 0; m < nterms; ++m) {
    const double* g = G + (long long)m * dim * n1d;
    double v = coef[m] * g[i0] * g[n1d + i1];
    if (dim == 3) v *= g[2 * n1d + i2];
    s += v;
  }
  b[idx] = (T)s;
}

// ------------------------------------------------------------------ L2 error

// Squared L2 error of u_h (nodal values x) against u = sum_m uc[m] prod_a sin(pi kappa_ma x_a)
// with cellwise nq^d Gauss points.  One thread per (cell, q2, q1) quadrature line: it contracts
// the (k+1)^d nodal values of its cell over axes 2 and 1 (V[q*(k+1) + i] = phi_i(xi_q)), then
// evaluates the nq points of the line along axis 0.  u comes from per-axis sine tables
// S[(m*dim + a)*ncells*nq + c*nq + q].  Block partial sums in a fixed order.
template <int K>
__global__ void __launch_bounds__(256) l2_error_kernel(const double* __restrict__ x, const double* __restrict__ V,
                                                       const double* __restrict__ wq, const double* __restrict__ S,
                                                       const double* __restrict__ uc, int nmodes, int dim, int nq,
                                                       long long ncells, long long n1d, long long nlines,
                                                       double cellvol, double* __restrict__ partial) {
  constexpr int NP = K + 1;
  __shared__ double red[256];
  double acc = 0.0;
  const long long nql = dim == 2 ? nq : (long long)nq * nq;  // lines per cell
  const long long na = ncells * nq;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nlines; t += (long long)gridDim.x * blockDim.x) {
    const long long cell = t / nql;
    const int li = (int)(t - cell * nql);
    const int q1 = li % nq, q2 = dim == 3 ? li / nq : 0;
    const long long c0 = cell % ncells, c1 = (cell / ncells) % ncells, c2 = dim == 3 ? cell / (ncells * ncells) : 0;
    const long long base = (dim == 3 ? (long long)K * c2 * n1d * n1d : 0) + (long long)K * c1 * n1d + (long long)K * c0;
    double line[NP];
#pragma unroll
    for (int i0 = 0; i0 < NP; ++i0) line[i0] = 0.0;
    for (int i2 = 0; i2 < (dim == 3 ? NP : 1); ++i2) {
      const double v2 = dim == 3 ? V[q2 * NP + i2] : 1.0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        const double v21 = v2 * V[q1 * NP + i1];
        const double* row = x + base + (long long)i2 * n1d * n1d + (long long)i1 * n1d;
#pragma unroll
        for (int i0 = 0; i0 < NP; ++i0) line[i0] = fma(v21, row[i0], line[i0]);
      }
    }
    double w12 = wq[q1] * cellvol;
    if (dim == 3) w12 *= wq[q2];
    for (int q0 = 0; q0 < nq; ++q0) {
      double uh = 0.0;
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) uh = fma(V[q0 * NP + i0], line[i0], uh);
      double u = 0.0;
      for (int m = 0; m < nmodes; ++m) {
        const double* Sm = S + (long long)m * dim * na;
        double v = uc[m] * Sm[c0 * nq + q0] * Sm[na + c1 * nq + q1];
        if (dim == 3) v *= Sm[2 * na + c2 * nq + q2];
        u += v;
      }
      const double e = u - uh;
      acc = fma(w12 * wq[q0] * e, e, acc);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ launchers

namespace {

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Workgroups the streaming operator aims for: 2048, except FP64 at degrees 4 and 7, where fewer,
// longer chunks measured faster (3D Q4 64^3 apply 101 -> 93 us with 1024, mixed solve -0.8%;
// Q7 32^3 210 -> 184 us with 512).  Degrees 2 and 3 measured slower that way, degree 5 equal and
// degree 6 gave a faster apply but a slower solve.
template <int K, typename T>
constexpr long long op_stream_target() {
  return sizeof(T) == 8 && K == 4 ? 1024 : sizeof(T) == 8 && K == 7 ? 512 : 2048;
}
template <int K, typename T>
long long op_stream_blocks(const LevelGeom& g, int* t0_out, int* cz_out) {
  using S = OpStream<K>;
  const int t0 = ceil_div(g.ncells, S::CX);
  // enough workgroups to fill the chip, chunks of at least 4 cells along x2
  const long long tiles = (long long)t0 * t0;
  const long long target = op_stream_target<K, T>();
  long long chunks = (target + tiles - 1) / tiles;
  if (chunks > g.ncells / 4) chunks = g.ncells / 4;
  if (chunks < 1) chunks = 1;
  const int cz = (int)((g.ncells + chunks - 1) / chunks);
  chunks = (g.ncells + cz - 1) / cz;
  *t0_out = t0;
  *cz_out = cz;
  return tiles * chunks;
}

// The streaming kernel addresses a cell's K node planes with byte offsets below 2^31 (bit 31 of its
// per-element offsets marks nodes outside the interior).
template <int K, typename T>
bool op_stream_fits(const LevelGeom& g) {
  return (long long)(K + 1) * g.n1d * g.n1d * (long long)sizeof(T) < (1LL << 31);
}

template <int K, typename T>
hipError_t op_stream_launch(const LevelGeom& g, const void* x, const void* b, void* y, hipStream_t st,
                            double* pq_part = nullptr) {
  using S = OpStream<K>;
  if (!op_stream_fits<K, T>(g)) return hipErrorInvalidConfiguration;
  int t0, cz;
  const long long blocks = op_stream_blocks<K, T>(g, &t0, &cz);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const T scale = (T)g.h;  // A_h = h A_1 in 3D
  if (b)
    hipLaunchKernelGGL((op_stream_kernel<K, T, true>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)x,
                       (const T*)b, (T*)y, g.n1d, t0, t0, cz, scale, pq_part);
  else
    hipLaunchKernelGGL((op_stream_kernel<K, T, false>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)x,
                       (const T*)nullptr, (T*)y, g.n1d, t0, t0, cz, scale, pq_part);
  return hipGetLastError();
}

// The tile kernel indexes with 64-bit node offsets; its grid (and tiles0 * tiles1 in int) must fit.
template <int D, int K>
bool op_tile_fits(const LevelGeom& g) {
  using S = OpShape<D, K>;
  const long long t0 = ceil_div(g.ncells, S::C0), t1 = ceil_div(g.ncells, S::C1),
                  t2 = D == 3 ? ceil_div(g.ncells, S::C2) : 1;
  return t0 * t1 <= 0x7fffffffLL && t0 * t1 * t2 <= 0x7fffffffLL;
}

template <int D, int K>
long long op_tile_blocks(const LevelGeom& g) {
  using S = OpShape<D, K>;
  return (long long)ceil_div(g.ncells, S::C0) * ceil_div(g.ncells, S::C1) * (D == 3 ? ceil_div(g.ncells, S::C2) : 1);
}

// pq_part != null (2D FP64 only): per-workgroup partial sums, see op_tile_kernel
template <int D, int K, typename T>
hipError_t op_tile_launch(const LevelGeom& g, const void* x, const void* b, void* y, hipStream_t st,
                          double* pq_part = nullptr) {
  using S = OpShape<D, K>;
  const int t0 = ceil_div(g.ncells, S::C0), t1 = ceil_div(g.ncells, S::C1);
  const long long blocks = op_tile_blocks<D, K>(g);
  if (!op_tile_fits<D, K>(g)) return hipErrorInvalidConfiguration;
  if (pq_part && (D != 2 || sizeof(T) != 8)) return hipErrorInvalidValue;
  const T scale = (T)(D == 3 ? g.h : 1.0);  // A_h = h^(d-2) A_1
  if (b)
    hipLaunchKernelGGL((op_tile_kernel<D, K, T, true>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)x,
                       (const T*)b, (T*)y, g.n1d, t0, t1, scale, pq_part);
  else
    hipLaunchKernelGGL((op_tile_kernel<D, K, T, false>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)x,
                       (const T*)nullptr, (T*)y, g.n1d, t0, t1, scale, pq_part);
  return hipGetLastError();
}

#ifndef VPS_OP_STREAM_MIN_CELLS
#define VPS_OP_STREAM_MIN_CELLS 32
#endif
constexpr long long kOpStreamMinCells = VPS_OP_STREAM_MIN_CELLS;

template <int D, int K, typename T>
hipError_t op_launch(const LevelGeom& g, const void* x, const void* b, void* y, hipStream_t st) {
  if constexpr (D == 3) {
    // small levels have too few column tiles to hide the plane-to-plane chain of the streaming
    // kernel: the cubic tiles run fully in parallel there
    if (g.ncells >= kOpStreamMinCells && op_stream_fits<K, T>(g)) return op_stream_launch<K, T>(g, x, b, y, st);
    return op_tile_launch<D, K, T>(g, x, b, y, st);
  } else {
    return op_tile_launch<D, K, T>(g, x, b, y, st);
  }
}

template <int D, int K>
bool pro_fits(const LevelGeom& fine) {
  const long long ncc = fine.ncells / 2;
  if (D == 3 && kPro3Tiles<K>) {
    using S = Pro3<K>;
    const long long t0 = ceil_div(ncc, S::C0), t1 = ceil_div(ncc, S::C1), t2 = ceil_div(ncc, S::C2);
    return t0 * t1 <= 0x7fffffffLL && t0 * t1 * t2 <= 0x7fffffffLL;
  }
  using S = ProShape<D, K>;
  const long long t0 = ceil_div(ncc, S::C0), t1 = ceil_div(ncc, S::C1);
  return t0 * t1 <= 0x7fffffffLL && t0 * t1 * (D == 3 ? t0 : 1) <= 0x7fffffffLL;
}

template <int D, int K, typename T>
hipError_t pro_launch(const LevelGeom& fine, const void* e, void* xf, hipStream_t st) {
  const long long ncc = fine.ncells / 2;
  const long long n1dc = (long long)K * ncc + 1;
  if (!pro_fits<D, K>(fine)) return hipErrorInvalidConfiguration;
  if (D == 3 && kPro3Tiles<K>) {
    using S = Pro3<K>;
    const int t0 = ceil_div(ncc, S::C0), t1 = ceil_div(ncc, S::C1), t2 = ceil_div(ncc, S::C2);
    const long long blocks = (long long)t0 * t1 * t2;
    hipLaunchKernelGGL((prolong3_kernel<K, T>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)e, (T*)xf, n1dc,
                       fine.n1d, t0, t1);
    return hipGetLastError();
  }
  using S = ProShape<D, K>;
  const int t0 = ceil_div(ncc, S::C0), t1 = ceil_div(ncc, S::C1);
  const long long blocks = (long long)t0 * t1 * (D == 3 ? t0 : 1);
  hipLaunchKernelGGL((prolong_tile_kernel<D, K, T>), dim3((unsigned)blocks), dim3(S::NT), 0, st, (const T*)e, (T*)xf,
                     n1dc, fine.n1d, t0, t1);
  return hipGetLastError();
}

// 3D: in-plane reduction of every fine plane, then the x2 reduction (scratch t: nf x nc x nc).
// 2D: x0 pass into t (nf x nc), then the x1 pass.
// The restriction's launch limits: 32-bit offsets inside the plane pass's group of fine planes and
// inside a coarse plane of the intermediate, grid dimensions y and z below 2^16, grids below 2^31.
template <int D, int K, typename T>
bool res_fits(const LevelGeom& fine) {
  const long long nf = fine.n1d, nc = K * (fine.ncells / 2) + 1, ncc = (nc - 1) / K;
  if (nf > 0x7fffffffLL) return false;
  if (D == 3) {
    using S = ResPlane<K, T>;
    const long long tiles = ceil_div(nc - 1, S::TX), groups = ceil_div(nf - 2, S::GP);
    return tiles * tiles <= 0x7fffffffLL && groups <= 65535 && S::GP * nf * nf * (long long)sizeof(T) < (1LL << 31) &&
           nc <= 65535 && ncc <= 65535 && nc * nc * (long long)sizeof(T) < (1LL << 32) &&
           ceil_div(ncc, kResCellsPerThread) <= 65535;
  }
  return ceil_div(nc, Res2D<K, T>::TX) * ceil_div(nc, Res2D<K, T>::TX) <= 0x7fffffffLL;
}

template <int D, int K, typename T>
hipError_t res_launch(const LevelGeom& fine, const void* rf, void* rc, hipStream_t st, void* t, void* xz) {
  const int nf = (int)fine.n1d, nc = (int)(K * (fine.ncells / 2) + 1);
  const int ncc = (nc - 1) / K;
  if (!res_fits<D, K, T>(fine)) return hipErrorInvalidConfiguration;
  if (D == 3) {
    using S = ResPlane<K, T>;
    // tiles cover coarse columns 0 .. nc - 2: the x2 pass writes 0 on the last column and row
    // whatever the plane values there are
    const int tiles = ceil_div(nc - 1, S::TX);
    const int groups = ceil_div(nf - 2, S::GP);
    hipLaunchKernelGGL((restrict_plane_kernel<K, T>), dim3((unsigned)(tiles * tiles), (unsigned)groups), dim3(S::NT),
                       0, st, (const T*)rf, (T*)t, (long long)nf, (long long)nc, tiles);
    hipLaunchKernelGGL((restrict_z_kernel<K, T>), dim3((unsigned)((nc + 63) / 64), (unsigned)((nc + 3) / 4),
                                                      (unsigned)ceil_div(ncc, kResCellsPerThread)),
                       dim3(64, 4), 0, st, (const T*)t, (T*)rc, nf, nc, (T*)xz);
  } else {
    const int tiles = ceil_div(nc, Res2D<K, T>::TX);
    hipLaunchKernelGGL((restrict_tile2d_kernel<K, T>), dim3((unsigned)(tiles * tiles)), dim3(Res2D<K, T>::NT), 0, st,
                       (const T*)rf, (T*)rc, (T*)xz, (long long)nf, (long long)nc, tiles);
  }
  return hipGetLastError();
}

}  // namespace

#define VPS_DISPATCH(FN, G, PREC, ...)                                                   \
  do {                                                                                   \
    const int d_ = (G).dim, k_ = (G).k;                                                  \
    switch (d_ * 100 + k_ * 10 + (PREC)) {                                               \
      case 210: return FN<2, 1, double>(G, __VA_ARGS__);                                 \
      case 211: return FN<2, 1, float>(G, __VA_ARGS__);                                  \
      case 220: return FN<2, 2, double>(G, __VA_ARGS__);                                 \
      case 221: return FN<2, 2, float>(G, __VA_ARGS__);                                  \
      case 230: return FN<2, 3, double>(G, __VA_ARGS__);                                 \
      case 231: return FN<2, 3, float>(G, __VA_ARGS__);                                  \
      case 240: return FN<2, 4, double>(G, __VA_ARGS__);                                 \
      case 241: return FN<2, 4, float>(G, __VA_ARGS__);                                  \
      case 250: return FN<2, 5, double>(G, __VA_ARGS__);                                 \
      case 251: return FN<2, 5, float>(G, __VA_ARGS__);                                  \
      case 260: return FN<2, 6, double>(G, __VA_ARGS__);                                 \
      case 261: return FN<2, 6, float>(G, __VA_ARGS__);                                  \
      case 270: return FN<2, 7, double>(G, __VA_ARGS__);                                 \
      case 271: return FN<2, 7, float>(G, __VA_ARGS__);                                  \
      case 310: return FN<3, 1, double>(G, __VA_ARGS__);                                 \
      case 311: return FN<3, 1, float>(G, __VA_ARGS__);                                  \
      case 320: return FN<3, 2, double>(G, __VA_ARGS__);                                 \
      case 321: return FN<3, 2, float>(G, __VA_ARGS__);                                  \
      case 330: return FN<3, 3, double>(G, __VA_ARGS__);                                 \
      case 331: return FN<3, 3, float>(G, __VA_ARGS__);                                  \
      case 340: return FN<3, 4, double>(G, __VA_ARGS__);                                 \
      case 341: return FN<3, 4, float>(G, __VA_ARGS__);                                  \
      case 350: return FN<3, 5, double>(G, __VA_ARGS__);                                 \
      case 351: return FN<3, 5, float>(G, __VA_ARGS__);                                  \
      case 360: return FN<3, 6, double>(G, __VA_ARGS__);                                 \
      case 361: return FN<3, 6, float>(G, __VA_ARGS__);                                  \
      case 370: return FN<3, 7, double>(G, __VA_ARGS__);                                 \
      case 371: return FN<3, 7, float>(G, __VA_ARGS__);                                  \
    }                                                                                    \
    return hipErrorInvalidValue;                                                         \
  } while (0)

namespace {

// Every operator and transfer launch the library issues on level g in precision T is accepted by
// its launcher: grids within their limits, the kernels' 32-bit offsets valid, tiles and chunks
// covering the level.
template <int D, int K, typename T>
bool grid_launches_ok(const LevelGeom& g, std::string* why) {
  const std::string tag = std::string(sizeof(T) == 8 ? "FP64 " : "FP32 ");
  if (D == 3 && g.ncells >= kOpStreamMinCells && op_stream_fits<K, T>(g)) {
    using S = OpStream<K>;
    int t0 = 0, cz = 0;
    const long long blocks = op_stream_blocks<K, T>(g, &t0, &cz);
    const long long tiles = (long long)t0 * t0, chunks = tiles > 0 ? blocks / tiles : 0;
    if (blocks > 0x7fffffffLL) return *why = tag + "streaming operator: grid too large", false;
    if ((long long)t0 * S::CX < g.ncells || chunks * cz < g.ncells)
      return *why = tag + "streaming operator: tiles or chunks do not cover the level", false;
  } else if (!op_tile_fits<D, K>(g)) {
    return *why = tag + "operator tiles: grid too large", false;
  }
  if (g.level >= 2) {
    if (!res_fits<D, K, T>(g)) return *why = tag + "restriction: launch limits exceeded", false;
    if (!pro_fits<D, K>(g)) return *why = tag + "prolongation: grid too large", false;
  }
  return true;
}

template <int D, int K>
bool grid_launches_both(const LevelGeom& g, std::string* why) {
  return grid_launches_ok<D, K, double>(g, why) && grid_launches_ok<D, K, float>(g, why);
}

}  // namespace

bool check_grid_launches(const LevelGeom& g, std::string* why) {
  switch (g.dim * 10 + g.k) {
    case 21: return grid_launches_both<2, 1>(g, why);
    case 22: return grid_launches_both<2, 2>(g, why);
    case 23: return grid_launches_both<2, 3>(g, why);
    case 24: return grid_launches_both<2, 4>(g, why);
    case 25: return grid_launches_both<2, 5>(g, why);
    case 26: return grid_launches_both<2, 6>(g, why);
    case 27: return grid_launches_both<2, 7>(g, why);
    case 31: return grid_launches_both<3, 1>(g, why);
    case 32: return grid_launches_both<3, 2>(g, why);
    case 33: return grid_launches_both<3, 3>(g, why);
    case 34: return grid_launches_both<3, 4>(g, why);
    case 35: return grid_launches_both<3, 5>(g, why);
    case 36: return grid_launches_both<3, 6>(g, why);
    case 37: return grid_launches_both<3, 7>(g, why);
  }
  *why = "unsupported (dim, degree)";
  return false;
}

hipError_t launch_operator(const LevelGeom& g, int prec, const void* x, const void* b, void* y, hipStream_t st) {
  VPS_DISPATCH(op_launch, g, prec, x, b, y, st);
}

namespace {
// out[0] = sum of part[0..n) in a fixed order (one workgroup of blockDim.x <= 1024 threads)
__global__ __launch_bounds__(1024) void sum_parts_kernel(const double* __restrict__ part, int n,
                                                          double* __restrict__ out) {
  __shared__ double red[1024];
  const int nt = blockDim.x, tid = threadIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int i = tid; i < n; i += nt) s += part[i];
  red[tid] = s;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[0] = red[0];
}

hipError_t sum_parts(const double* part, long long n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(n > 4096 ? 1024 : 256), 0, st, part, (int)n, out);
  return hipGetLastError();
}

// Partial sums the fused forms take on level g (0: no fused form there).  3D: the streaming
// operator on levels that it serves; 2D: the tile operator.
template <int K>
long long fused_parts_k(const LevelGeom& g) {
  if (g.dim == 3) {
    if (g.ncells < kOpStreamMinCells || !op_stream_fits<K, double>(g)) return 0;
    int t0, cz;
    return op_stream_blocks<K, double>(g, &t0, &cz);
  }
  if (!op_tile_fits<2, K>(g)) return 0;
  return op_tile_blocks<2, K>(g);
}

long long fused_parts(const LevelGeom& g) {
  switch (g.k) {
    case 1: return fused_parts_k<1>(g);
    case 2: return fused_parts_k<2>(g);
    case 3: return fused_parts_k<3>(g);
    case 4: return fused_parts_k<4>(g);
    case 5: return fused_parts_k<5>(g);
    case 6: return fused_parts_k<6>(g);
    case 7: return fused_parts_k<7>(g);
  }
  return 0;
}

// x, b: the operator's input and right-hand side (b null: y = A x with x.y partials; b set: |b - A x|^2
// partials, y not written)
template <int K>
hipError_t fused_op_k(const LevelGeom& g, const double* x, const double* b, double* y, double* part,
                      hipStream_t st) {
  if (g.dim == 3) return op_stream_launch<K, double>(g, x, b, y, st, part);
  return op_tile_launch<2, K, double>(g, x, b, y, st, part);
}

hipError_t fused_op(const LevelGeom& g, const double* x, const double* b, double* y, double* part, long long max_parts,
                    double* out, hipStream_t st, bool* fused) {
  *fused = false;
  const long long n = fused_parts(g);
  // no fused form, or more partial sums than the buffer holds: the caller takes the unfused path
  if (n <= 0 || n > max_parts) return hipSuccess;
  hipError_t e = hipErrorInvalidValue;
  switch (g.k) {
    case 1: e = fused_op_k<1>(g, x, b, y, part, st); break;
    case 2: e = fused_op_k<2>(g, x, b, y, part, st); break;
    case 3: e = fused_op_k<3>(g, x, b, y, part, st); break;
    case 4: e = fused_op_k<4>(g, x, b, y, part, st); break;
    case 5: e = fused_op_k<5>(g, x, b, y, part, st); break;
    case 6: e = fused_op_k<6>(g, x, b, y, part, st); break;
    case 7: e = fused_op_k<7>(g, x, b, y, part, st); break;
  }
  if (e != hipSuccess) return e;
  e = sum_parts(part, n, out, st);
  if (e == hipSuccess) *fused = true;
  return e;
}
}  // namespace

long long fused_reduction_parts(const LevelGeom& g) { return fused_parts(g); }

hipError_t launch_residual_norm2(const LevelGeom& g, const double* x, const double* b, double* part,
                                 long long max_parts, double* out, hipStream_t st, bool* fused) {
  return fused_op(g, x, b, nullptr, part, max_parts, out, st, fused);
}

hipError_t launch_operator_pq(const LevelGeom& g, const double* p, double* q, double* part, long long max_parts,
                              double* out, hipStream_t st, bool* fused) {
  return fused_op(g, p, nullptr, q, part, max_parts, out, st, fused);
}

hipError_t launch_prolongate_add(const LevelGeom& fine, int prec, const void* e, void* xf, hipStream_t st) {
  VPS_DISPATCH(pro_launch, fine, prec, e, xf, st);
}

hipError_t launch_restrict(const LevelGeom& fine, int prec, const void* rf, void* rc, void* t, hipStream_t st,
                           void* xc_zero) {
  VPS_DISPATCH(res_launch, fine, prec, rf, rc, st, t, xc_zero);
}

// ------------------------------------------- scratch of the allocation-free restriction
//
// One array per GPU, held from the module's load until the process ends.  Its name is a host-side
// stand-in: host code passes only the device address looked up per device below.  Every call on a
// GPU shares that GPU's array (calls that overlap on one GPU race); the restriction writes every
// scratch entry it later uses, so nothing needs clearing between calls.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device ordinal
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // with this device current
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_zero_boundary(const LevelGeom& g, int prec, void* y, hipStream_t st) {
  const long long faces = g.dim == 2 ? g.n1d : g.n1d * g.n1d;
  const unsigned blocks = (unsigned)((faces + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(zero_boundary_kernel<double>, dim3(blocks), dim3(256), 0, st, (double*)y, g.dim, g.n1d);
  else
    hipLaunchKernelGGL(zero_boundary_kernel<float>, dim3(blocks), dim3(256), 0, st, (float*)y, g.dim, g.n1d);
  return hipGetLastError();
}

hipError_t launch_rhs_separable(const LevelGeom& g, int prec, int nterms, const double* G, const double* coef, void* b,
                                hipStream_t st) {
  long long ntot = 1;
  for (int a = 0; a < g.dim; ++a) ntot *= g.n1d;
  const unsigned blocks = (unsigned)((ntot + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(rhs_separable_kernel<double>, dim3(blocks), dim3(256), 0, st, (double*)b, G, coef, nterms,
                       g.dim, g.n1d, ntot);
  else
    hipLaunchKernelGGL(rhs_separable_kernel<float>, dim3(blocks), dim3(256), 0, st, (float*)b, G, coef, nterms, g.dim,
                       g.n1d, ntot);
  return hipGetLastError();
}

hipError_t launch_l2_error(const LevelGeom& g, const double* x, const double* V, const double* wq, const double* S,
                           const double* uc, int nmodes, int nq, double* partial, int nparts, hipStream_t st) {
  const long long ncd = g.dim == 2 ? g.ncells * g.ncells : g.ncells * g.ncells * g.ncells;
  const long long nlines = ncd * (g.dim == 2 ? nq : nq * nq);
  const double cellvol = g.dim == 2 ? g.h * g.h : g.h * g.h * g.h;
  switch (g.k) {
#define VPS_L2(KK)                                                                                                 \
  case KK:                                                                                                         \
    hipLaunchKernelGGL(l2_error_kernel<KK>, dim3(nparts), dim3(256), 0, st, x, V, wq, S, uc, nmodes, g.dim, nq,    \
                       g.ncells, g.n1d, nlines, cellvol, partial);                                                   \
    break;
    VPS_L2(1) VPS_L2(2) VPS_L2(3) VPS_L2(4) VPS_L2(5) VPS_L2(6) VPS_L2(7)
#undef VPS_L2
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


}  // namespace vps
