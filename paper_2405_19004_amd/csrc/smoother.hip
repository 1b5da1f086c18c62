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
// Boundary mode (Sec. 4.1.3, eq:A_ib_2d/3d) uses that the local solver is exact:
//   x_j^I <- A_j^{-1} (b_j^I - A^{IB} x_j^B),
// i.e. the residual is formed with the patch interior taken as zero and the
// interior is overwritten, so x^I is never loaded.
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
#include "patch_tables_gen.hpp"

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
// Degrees (bit K) whose 2D shape takes one wave (64 threads, half the patches) instead of two:
// measured 1-3% faster per V-cycle at degrees 3, 4, 5 and 7, equal at 2 and 6, slower at 1.
#ifndef VPS_2D_WAVE_MASK
#define VPS_2D_WAVE_MASK 0xB8
#endif
template <int K> struct SmootherShape<2, K> {
  static constexpr bool ONE_WAVE = ((VPS_2D_WAVE_MASK) >> K) & 1;
  static constexpr int PPW = (K == 1 ? 64 : K == 2 ? 32 : K == 3 ? 16 : K <= 5 ? 12 : 8) / (ONE_WAVE ? 2 : 1);
  static constexpr int NT = ONE_WAVE ? 64 : 128;
};
#ifndef VPS_Q4_3D_PPW
#define VPS_Q4_3D_PPW 2
#endif
#ifndef VPS_Q4_3D_NT
#define VPS_Q4_3D_NT 128
#endif
// Degrees (bit K) whose default 3D shape takes the aliased LDS layout: measured 2-13% faster for
// degrees 3-7 (occupancy), no gain for degrees 1-2, where the layout is already small.
#ifndef VPS_3D_ALIAS_MASK
#define VPS_3D_ALIAS_MASK 0xF8
#endif
template <int K> struct SmootherShape<3, K> {
  static constexpr int PPW = K == 1 ? 32 : K == 2 ? 8 : K == 3 ? 4 : K == 4 ? VPS_Q4_3D_PPW : 1;
  static constexpr int NT = K == 4 ? VPS_Q4_3D_NT : K <= 5 ? 128 : K == 6 ? 192 : 256;
  // the default shape of the multiplicative pass shares one LDS region between the closure and the
  // first two contraction stages (see SmootherLds)
  static constexpr bool ALIAS = ((VPS_3D_ALIAS_MASK) >> K) & 1;
};

// Patches per workgroup for small launches (coarse levels): fewer patches per workgroup means
// fewer tasks per thread in every stage, so a workgroup finishes sooner; used when the default
// shape would give fewer than kLatencyBlocks workgroups, where the chip is not full anyway.
template <int D, int K>
struct LatencyPPW {
  static constexpr int value = D == 3 ? (K == 1 ? 8 : K == 2 ? 2 : 1) : (K == 1 ? 16 : K == 2 ? 8 : K <= 5 ? 4 : 2);
};
#ifndef VPS_LATENCY_BLOCKS
#define VPS_LATENCY_BLOCKS 1024
#endif
constexpr long long kLatencyBlocks = VPS_LATENCY_BLOCKS;

// Two words of T moved by one 8- or 16-byte LDS access.
template <typename T>
struct Pair;
template <>
struct Pair<float> {
  using type = float2;
};
template <>
struct Pair<double> {
  using type = double2;
};

// Smallest s >= v with s = r (mod 32): padded outer strides of the LDS transpose buffers.
constexpr int pad32(int v, int r) { return v + ((r - v) % 32 + 32) % 32; }

// LDS layouts.  Every transpose buffer puts the loop axis of the stage that reads it outermost,
// so the reading lanes touch consecutive words; the outer stride is padded (mod 32) so that the
// writing lanes of the previous stage also fall into distinct banks.
template <int D, int K, typename T, bool ADD, int PPWv, bool ALIASv = false, bool PAIRv = false>
struct SmootherLds {
  static constexpr int n = 2 * K + 1, m = 2 * K - 1;
  static constexpr int PPW = PPWv;
  static constexpr int RS = 2 * K * PPW + 1;  // closure row segment of the workgroup
  // ---- 3D strides
  // residue of the P stride that makes the x0-contraction writes conflict-free (searched per degree
  // for the launch shapes above, 4- and 8-byte words)
  static constexpr int kSJ1Res[8] = {0, 11, 7, 19, 15, 27, 23, 3};
  static constexpr int SJ1 = pad32(PPW * n * m, kSJ1Res[K]);  // P  [j1][q][j2][i0]   (PM, PA)
  static constexpr int SJ2 = pad32(PPW * m * m, m);          // UV [j2][q][i1][i0]   (U, V)
  static constexpr int SI1 = pad32(PPW * m * m, m);          // W4 [i1][q][a2][i0]
  static constexpr int SI0 = pad32(PPW * m * m, 1);          // W5 [i0][q][a2][a1]
  static constexpr int SA1 = pad32(PPW * m * m, 1);          // W6 [a1][q][a2][i0]
  static constexpr int SA2 = pad32(PPW * m * m, m);          // W7 [a2][q][i1][i0]
  static constexpr int X3 = ADD ? 0 : n * n * RS;
  static constexpr int P3 = ADD ? 0 : 2 * n * SJ1;
  static constexpr int UV3 = ADD ? 0 : 2 * n * SJ2;
  static constexpr int A3 = P3 > m * SI1 ? (P3 > m * SA1 ? P3 : m * SA1) : (m * SI1 > m * SA1 ? m * SI1 : m * SA1);
  static constexpr int B3a = X3 > UV3 ? X3 : UV3;
  static constexpr int B3b = m * SI0 > m * SA2 ? m * SI0 : m * SA2;
  static constexpr int B3 = B3a > B3b ? B3a : B3b;
  // ---- 2D strides
  static constexpr int T1 = pad32(PPW * m, (m * PPW) % 32);  // P2  [j1][q][i0]  (PM, PA)
  static constexpr int T0 = pad32(PPW * m, 1);               // W   [i0][q][a1]
  static constexpr int TA = pad32(PPW * m, 1);               // W2  [a1][q][i0]
  static constexpr int X2 = ADD ? 0 : n * RS;
  static constexpr int P2 = ADD ? 0 : 2 * n * T1;
  static constexpr int A2 = P2 > m * TA ? P2 : m * TA;
  static constexpr int B2 = X2 > m * T0 ? X2 : m * T0;
  // ---- aliased 3D layout (multiplicative): the closure X, PM/PA and U/V all start at word 0 (the x0
  // and x1 stages read their inputs into registers and the workgroup synchronises before they
  // write), the x2 and x0 diagonalisation outputs (W4, W6) follow U/V, the x1 ones (W5, W7) start
  // at 0 again once U/V is dead
  static constexpr bool AL = ALIASv && D == 3 && !ADD;
  static constexpr int W46 = m * SI1 > m * SA1 ? m * SI1 : m * SA1;
  static constexpr int W57 = m * SI0 > m * SA2 ? m * SI0 : m * SA2;
  static constexpr int AL3a = X3 > P3 ? X3 : P3;
  static constexpr int AL3 = AL3a > UV3 + W46 ? AL3a : UV3 + W46;
  // ---- paired 3D layout (aliased, smaller still): PM and PA interleaved as pairs [j1][q][j2][i0]{M, A}
  // (one 8-byte access per pair, the pair stride SJP padded for conflict-free writes of the x0
  // stage), W4 also over U/V (the x2 stage synchronises before it writes), W5 and W7 after W4/W6
  static constexpr bool PR = PAIRv && AL;
  static constexpr int SJP = pad32(2 * PPW * n * m, 30);
  static constexpr int PP3 = ADD ? 0 : n * SJP;
  static constexpr int PR3a = X3 > PP3 ? X3 : PP3;
  static constexpr int PR3b = UV3 > W46 + W57 ? UV3 : W46 + W57;
  static constexpr int PR3 = PR3a > PR3b ? PR3a : PR3b;
  // ---- aliased 2D layout (multiplicative): X, PM/PA and the x1 stage's output W start at word 0
  // (the x0 and x1 stages compute every line, the workgroup synchronises, then they write over
  // their inputs); W2 follows W
  static constexpr bool AL2 = ALIASv && D == 2 && !ADD;
  static constexpr int AL2a = X2 > P2 ? X2 : P2;
  static constexpr int AL2T = AL2a > m * T0 + m * TA ? AL2a : m * T0 + m * TA;
  static constexpr int total = D == 3 ? (PR ? PR3 : AL ? AL3 : A3 + B3) : (AL2 ? AL2T : A2 + B2);
  static constexpr int offX2 = AL2 ? 0 : A2, offP2 = 0, offW = AL2 ? 0 : A2, offW2 = AL2 ? m * T0 : 0;
  // 3D buffers
  static constexpr int offX = AL ? 0 : A3;
  static constexpr int offP = 0;
  static constexpr int offUV = AL ? 0 : A3;
  static constexpr int offW46 = PR ? 0 : AL ? UV3 : 0;  // W4 and W6
  static constexpr int offW57 = PR ? W46 : AL ? 0 : A3;  // W5 and W7
};

__device__ __forceinline__ bool on_boundary(long long i, long long n1d) { return i == 0 || i == n1d - 1; }

// A per-lane LDS offset the optimiser may not take apart.  Without it, base + i * stride inside an
// unrolled loop is re-associated into a fresh (quarter-rate) 32-bit multiply per element; behind
// this barrier each element is the base register plus a constant in the instruction's offset field.
__device__ __forceinline__ int lds_base(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The constant tables re-derived through an opaque (but wave-uniform) zero
// offset: keeps the compiler from hoisting every table load out of a stage's
// task loop, which would pin more values in SGPRs than exist and spill them.
template <typename T>
__device__ __forceinline__ const DevTables<T>& tab_fresh(int k) {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return *reinterpret_cast<const DevTables<T>*>(reinterpret_cast<const char*>(&tab<T>(k)) + z);
}

// Eigenvector applications with the mirror parity of the patch eigenvectors (the 1D patch pair
// is symmetric under i -> m-1-i, so S[m-1-i][a] = par[a] S[i][a]): an even vector only sees
// v_i + v_{m-1-i}, an odd one v_i - v_{m-1-i}, which halves the multiply-adds.
// t[a] = sum_i S[i][a] v[i]
template <typename T, int K>
__device__ __forceinline__ void apply_st(const T (&v)[2 * K - 1], T (&t)[2 * K - 1]) {
  using PT = gen::PatchTables<T, K>;
  constexpr int m = 2 * K - 1, h = K - 1;
  T e[K], o[K];
#pragma unroll
  for (int i = 0; i < h; ++i) {
    e[i] = v[i] + v[m - 1 - i];
    o[i] = v[i] - v[m - 1 - i];
  }
  e[h] = v[h];
#pragma unroll
  for (int a = 0; a < m; ++a) {
    T s = T(0);
    if (PT::par[a] > 0) {
#pragma unroll
      for (int i = 0; i <= h; ++i) s = fma_tab(PT::S[i * m + a], e[i], s);
    } else {
#pragma unroll
      for (int i = 0; i < h; ++i) s = fma_tab(PT::S[i * m + a], o[i], s);
    }
    t[a] = s;
  }
}

// w[i] = sum_a S[i][a] t[a]: w_i = E_i + O_i and w_{m-1-i} = E_i - O_i with E (O) the even (odd) part
template <typename T, int K>
__device__ __forceinline__ void apply_s(const T (&t)[2 * K - 1], T (&w)[2 * K - 1]) {
  using PT = gen::PatchTables<T, K>;
  constexpr int m = 2 * K - 1, h = K - 1;
#pragma unroll
  for (int i = 0; i <= h; ++i) {
    T ev = T(0), od = T(0);
#pragma unroll
    for (int a = 0; a < m; ++a) {
      if (PT::par[a] > 0) {
        ev = fma_tab(PT::S[i * m + a], t[a], ev);
      } else if (i < h) {
        od = fma_tab(PT::S[i * m + a], t[a], od);
      }
    }
    w[i] = i < h ? ev + od : ev;  // the middle row has no odd part
    if (i < h) w[m - 1 - i] = ev - od;
  }
}

// Degrees (bit K) whose FP64 3D multiplicative pass takes the aliased LDS layout below: measured
// 11-45% faster for degrees 2-7 (occupancy: 3D Q4 goes from 33 to 17 KB of LDS, from 8 to 18 waves
// per compute unit), equal at degree 1.
#ifndef VPS_MULT3_ALIAS_MASK
#define VPS_MULT3_ALIAS_MASK 0xFC
#endif

// LDS of the 3D multiplicative pass below (T words).  Buffer A holds PM, PA [i2][j1][c], later the
// results of stages C and E; buffer B holds U, V, later those of D and F.  Every transpose buffer
// after PM/PA is laid out [loop index of the reading stage][reading task], the outer stride padded
// (mod 32) so that the writing lanes also touch distinct banks: for U, V and the D->E buffer the
// residue was searched per degree with a bank model of both sides (4- and 8-byte words); the others
// are distinct by construction.
template <int K, int PPW>
struct Mult3Lds {
  static constexpr int n = 2 * K + 1, m = 2 * K - 1, mm = m * m;
  static constexpr int RS = 2 * K * PPW + 1;  // closure columns of the workgroup along x0
  static constexpr int PM = m * n * RS;       // one of PM, PA
  static constexpr int kSURes[8] = {0, 11, 7, 19, 15, 27, 23, 3};
  static constexpr int SU = pad32(PPW * mm, kSURes[K]);  // U, V  [j1][q][i2][i0]
  static constexpr int SW = pad32(PPW * mm, m);          // C->D  [i2][q][a1][i0]
  static constexpr int kSW2Res[8] = {0, 0, 3, 13, 23, 25, 3, 5};
  static constexpr int SW2 = pad32(PPW * mm, kSW2Res[K]); // D->E  [i0][q][a2][a1]
  static constexpr int SW3 = pad32(PPW * mm, 1);         // E->F  [a1][q][a2][i0]
  static constexpr int SW4 = pad32(PPW * mm, m);         // F->G  [a2][q][i1][i0]
  static constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
  static constexpr int A = max3(2 * PM, m * SW, m * SW3);
  static constexpr int B = max3(2 * n * SU, m * SW2, m * SW4);
  // Aliased layout: PM/PA, U/V and the C->D buffer all start at word 0 (stages B and C compute
  // every line, the workgroup synchronises, then they write over their inputs); the D->E and F->G
  // buffers follow the larger of C->D and E->F, which starts at 0 again.
  static constexpr bool AL = ((VPS_MULT3_ALIAS_MASK) >> K) & 1;
  static constexpr int X1 = m * SW > m * SW3 ? m * SW : m * SW3;
  static constexpr int ALT = max3(2 * PM, 2 * n * SU, X1 + (m * SW2 > m * SW4 ? m * SW2 : m * SW4));
  static constexpr int total = AL ? ALT : A + B;
  static constexpr int offP = 0, offUV = AL ? 0 : A;
  static constexpr int offW = 0, offW2 = AL ? X1 : A, offW3 = 0, offW4 = AL ? X1 : A;
};

// 3D multiplicative colour pass, closure contracted along x2 first.  Every thread of stage A loads
// one closure column along x2 straight from global memory and contracts it in registers, so the
// closure itself never goes through LDS.  Stages (lines, the axis contracted):
//   A  columns (j1, c)    x2: PM = M2 x, PA = A2 x                         -> A [i2][j1][c]
//   B  lines (q, i2, j1)  x0: U = M0 PM, V = A0 PM + M0 PA                  -> B [j1][q][i2][i0]
//   C  lines (q, i2, i0)  x1: r = b - h (A1 U + M1 V), then S^T along x1    -> A [i2][q][a1][i0]
//   D  lines (q, a1, i0)  S^T along x2                                      -> B [i0][q][a2][a1]
//   E  lines (q, a2, a1)  S^T along x0, 1/(lam2 + lam1 + lam0), S along x0  -> A [a1][q][a2][i0]
//   F  lines (q, a2, i0)  S along x1                                        -> B [a2][q][i1][i0]
//   G  lines (q, i1, i0)  S along x2, x^I += correction / h
// The three terms of the patch operator are those of the other contraction order up to rounding
// (1D factors on different axes commute).  b is read on the x1 lines of stage C; the update runs on
// the x2 lines of stage G, whose lanes share one node plane per access, and takes the old x^I from
// the thread's own stage A column.
template <int K, typename T, int PPW>
__device__ __forceinline__ void colour_pass_mult3(T* __restrict__ smem, const T* __restrict__ b, T* __restrict__ x,
                                                  long long n1d, int p0, int p1, int p2, int cnt0, int cnt1,
                                                  int groups0, T res_scale, T sol_scale, unsigned blk) {
  constexpr int n = 2 * K + 1, m = 2 * K - 1, mm = m * m;
  constexpr int NT = SmootherShape<3, K>::NT;
  using PT = gen::PatchTables<T, K>;
  using L = Mult3Lds<K, PPW>;
  constexpr int RS = L::RS;

  const ColourBlock cb = colour_block<3, K, PPW>(blk, p0, p1, p2, cnt0, cnt1, groups0);
  const int P = cb.count;
  const long long s0 = cb.s0, s1 = cb.s1, s2 = cb.s2;
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x;
  const int seg = 2 * K * P + 1;  // valid closure columns along x0
  // byte offsets inside the workgroup's closure fit in 32 bits (checked by the launcher)
  const int ld1 = (int)n1d;
  T* xo = x + (s2 * n1d2 + s1 * n1d + s0);  // closure corner of the first patch
  const T* bo = b + (s2 * n1d2 + s1 * n1d + s0);

  // b on the x1 lines (q, i2, i0) of stage C, prefetched now (tasks past the last patch are clamped
  // to it, so every load is in bounds); xpre is filled by stage A
  constexpr int NB = PPW * mm;
  constexpr int RB = (NB + NT - 1) / NT;
  T bpre[RB][m], xpre[RB][m];
  unsigned xoff[RB];  // byte offset of node (0, 1 + i1, 1 + i0) of stage G's line from the corner
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    int q = task / mm;
    const int r = task - q * mm;
    const int hi = r / m, lo = r - hi * m;  // (i2, i0) for stage C, (i1, i0) for stage G
    q = min(q, P - 1);
    const unsigned boff = (unsigned)(((1 + hi) * n1d2 + 2 * K * q + 1 + lo) * (long long)sizeof(T));
    xoff[rr] = (unsigned)(((1 + hi) * n1d + 2 * K * q + 1 + lo) * (long long)sizeof(T));
#pragma unroll
    for (int i = 0; i < m; ++i) bpre[rr][i] = ld_lane(bo + (1 + i) * ld1, boff);
  }

  // ---- A: closure columns along x2 -> PM, PA.  Tasks 0 .. NB-1 are the patch-interior columns in
  //      the order of stage G's lines (q, i1, i0), so a thread keeps the old x^I of its stage G line
  //      from its own column; the face columns (j1 on the closure boundary, or c on a patch
  //      boundary) follow.  Dirichlet nodes count as 0 (the boundary entries of x are not read as
  //      values).
  {
    T* PM = smem + L::offP;
    T* PA = PM + L::PM;
    constexpr int NF = 2 * RS + (n - 2) * (PPW + 1);  // face columns
    constexpr int NA = NB + NF;
    const bool lo0 = s0 == 0, hi0 = s0 + seg - 1 == n1d - 1;
    const bool lo1 = s1 == 0, hi1 = s1 + n - 1 == n1d - 1;
    const bool lo2 = s2 == 0, hi2 = s2 + n - 1 == n1d - 1;
#pragma unroll
    for (int it = 0; it < (NA + NT - 1) / NT; ++it) {
      const int t = it * NT + tid;
      int j1, c;
      if (t < NB) {
        const int q = t / mm, r = t - q * mm, i1 = r / m;
        j1 = 1 + i1;
        c = 2 * K * q + 1 + (r - i1 * m);
      } else {
        const int f = t - NB;
        if (f < 2 * RS) {
          j1 = f < RS ? 0 : n - 1;
          c = f < RS ? f : f - RS;
        } else {
          const int g = f - 2 * RS, jj = g / (PPW + 1);
          j1 = 1 + jj;
          c = 2 * K * (g - jj * (PPW + 1));
        }
      }
      if (t < NA && c < seg) {
        const unsigned off = (unsigned)(j1 * ld1 + c) * (unsigned)sizeof(T);
        T v[n];
#pragma unroll
        for (int j = 0; j < n; ++j) v[j] = ld_lane(xo + j * n1d2, off);
        if (it < RB && t < NB) {  // patch-interior column: never a Dirichlet node
#pragma unroll
          for (int i = 0; i < m; ++i) xpre[it < RB ? it : 0][i] = v[1 + i];
        }
        const bool zc = (c == 0 && lo0) || (c == seg - 1 && hi0) || (j1 == 0 && lo1) || (j1 == n - 1 && hi1);
        if (zc) {
#pragma unroll
          for (int j = 0; j < n; ++j) v[j] = T(0);
        }
        if (lo2) v[0] = T(0);
        if (hi2) v[n - 1] = T(0);
        const int o = lds_base(j1 * RS + c);
#pragma unroll
        for (int i = 0; i < m; ++i) {
          T sm = T(0), sa = T(0);
#pragma unroll
          for (int j = 0; j < n; ++j) {
            sm = fma_tab(PT::Mc[i * n + j], v[j], sm);
            sa = fma_tab(PT::Ac[i * n + j], v[j], sa);
          }
          PM[o + i * n * RS] = sm;
          PA[o + i * n * RS] = sa;
        }
      }
    }
  }
  __syncthreads();
  // ---- B: x0 lines (q, i2, j1), j1 fastest -> U, V
  {
    const T* PM = smem + L::offP;
    const T* PA = PM + L::PM;
    T* U = smem + L::offUV;
    T* V = U + n * L::SU;
    // x0 line of a task: U and V rows into su, sv; false past the workgroup's patches
    auto line = [&](int task, T* su, T* sv) -> bool {
      const int q = task / (m * n), r = task - q * (m * n);
      const int i2 = r / n, j1 = r - i2 * n;
      if (task >= PPW * m * n || q >= P) return false;
      const int ri = lds_base((i2 * n + j1) * RS + 2 * K * q);
      T pm[n], pa[n];
#pragma unroll
      for (int c = 0; c < n; ++c) {
        pm[c] = PM[ri + c];
        pa[c] = PA[ri + c];
      }
#pragma unroll
      for (int i = 0; i < m; ++i) {
        T au = T(0), av = T(0);
#pragma unroll
        for (int c = 0; c < n; ++c) {
          au = fma_tab(PT::Mc[i * n + c], pm[c], au);
          av = fma_tab(PT::Ac[i * n + c], pm[c], av);
          av = fma_tab(PT::Mc[i * n + c], pa[c], av);
        }
        su[i] = au;
        sv[i] = av;
      }
      return true;
    };
    auto put = [&](int task, const T* su, const T* sv) {
      const int q = task / (m * n), r = task - q * (m * n);
      const int i2 = r / n, j1 = r - i2 * n;
      const int o = lds_base(j1 * L::SU + (q * m + i2) * m);
#pragma unroll
      for (int i = 0; i < m; ++i) {
        U[o + i] = su[i];
        V[o + i] = sv[i];
      }
    };
    if constexpr (L::AL) {
      // U/V overwrite PM/PA: every line first, then the writes
      constexpr int RB2 = (PPW * m * n + NT - 1) / NT;
      T su[RB2][m], sv[RB2][m];
      bool ok[RB2];
#pragma unroll
      for (int rr = 0; rr < RB2; ++rr) ok[rr] = line(rr * NT + tid, su[rr], sv[rr]);
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < RB2; ++rr)
        if (ok[rr]) put(rr * NT + tid, su[rr], sv[rr]);
    } else {
      for (int base = 0; base < PPW * m * n; base += NT) {
        T su[m], sv[m];
        if (line(base + tid, su, sv)) put(base + tid, su, sv);
      }
    }
  }
  __syncthreads();
  // ---- C: x1 lines (q, i2, i0): residual, then S^T along x1.  Aliased layout: the C->D buffer
  //      overwrites U/V, so every line is computed before the workgroup synchronises and writes.
  T tc[RB][m];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    const int q = task / mm;
    if (task < NB && q < P) {
      const T* U = smem + L::offUV;
      const T* V = U + n * L::SU;
      T u[n], v[n];
#pragma unroll
      for (int j = 0; j < n; ++j) {
        u[j] = U[j * L::SU + task];
        v[j] = V[j * L::SU + task];
      }
      T res[m];
#pragma unroll
      for (int i = 0; i < m; ++i) {
        T sres = T(0);
#pragma unroll
        for (int j = 0; j < n; ++j) {
          sres = fma_tab(PT::Ac[i * n + j], u[j], sres);
          sres = fma_tab(PT::Mc[i * n + j], v[j], sres);
        }
        res[i] = fma(-res_scale, sres, bpre[rr][i]);
      }
      apply_st<T, K>(res, tc[rr]);
    }
  }
  if constexpr (L::AL) __syncthreads();
  {
    T* W = smem + L::offW;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / mm;
      if (task < NB && q < P) {
        const int r = task - q * mm, i2 = r / m, i0 = r - i2 * m;
        const int o = lds_base(i2 * L::SW + q * mm + i0);
#pragma unroll
        for (int a = 0; a < m; ++a) W[o + a * m] = tc[rr][a];
      }
    }
  }
  __syncthreads();
  // ---- D: x2 lines (q, a1, i0): S^T along x2
  for (int base = 0; base < PPW * mm; base += NT) {
    const int task = base + tid;
    const int q = task / mm;
    if (task < PPW * mm && q < P) {
      const T* W = smem + L::offW;
      T* W2 = smem + L::offW2;
      const int r = task - q * mm, a1 = r / m, i0 = r - a1 * m;
      T in[m];
#pragma unroll
      for (int i = 0; i < m; ++i) in[i] = W[i * L::SW + task];
      T t[m];
      apply_st<T, K>(in, t);
      const int o = lds_base(i0 * L::SW2 + q * mm + a1);
#pragma unroll
      for (int a = 0; a < m; ++a) W2[o + a * m] = t[a];
    }
  }
  __syncthreads();
  // ---- E: x0 lines (q, a2, a1): S^T along x0, eigenvalue scaling, S along x0
  for (int base = 0; base < PPW * mm; base += NT) {
    const int task = base + tid;
    const int q = task / mm;
    if (task < PPW * mm && q < P) {
      const T* W2 = smem + L::offW2;
      T* W3 = smem + L::offW3;
      const DevTables<T>& tb = tab_fresh<T>(K);
      const int r = task - q * mm, a2 = r / m, a1 = r - a2 * m;
      T in[m], z[m];
#pragma unroll
      for (int i = 0; i < m; ++i) in[i] = W2[i * L::SW2 + task];
      apply_st<T, K>(in, z);
#pragma unroll
      for (int a = 0; a < m; ++a) z[a] *= tb.inv3[r * m + a];
      T w[m];
      apply_s<T, K>(z, w);
      const int o = lds_base(a1 * L::SW3 + q * mm + a2 * m);
#pragma unroll
      for (int i = 0; i < m; ++i) W3[o + i] = w[i];
    }
  }
  __syncthreads();
  // ---- F: x1 lines (q, a2, i0): S along x1
  for (int base = 0; base < PPW * mm; base += NT) {
    const int task = base + tid;
    const int q = task / mm;
    if (task < PPW * mm && q < P) {
      const T* W3 = smem + L::offW3;
      T* W4 = smem + L::offW4;
      const int r = task - q * mm, a2 = r / m, i0 = r - a2 * m;
      T in[m];
#pragma unroll
      for (int a = 0; a < m; ++a) in[a] = W3[a * L::SW3 + task];
      T w[m];
      apply_s<T, K>(in, w);
      const int o = lds_base(a2 * L::SW4 + q * mm + i0);
#pragma unroll
      for (int i = 0; i < m; ++i) W4[o + i * m] = w[i];
    }
  }
  __syncthreads();
  // ---- G: x2 lines (q, i1, i0): S along x2 and x^I += correction, straight to global
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    const int q = task / mm;
    if (task < NB && q < P) {
      const T* W4 = smem + L::offW4;
      T in[m];
#pragma unroll
      for (int a = 0; a < m; ++a) in[a] = W4[a * L::SW4 + task];
      T w[m];
      apply_s<T, K>(in, w);
#pragma unroll
      for (int i = 0; i < m; ++i) st_lane(xo + (1 + i) * n1d2, xoff[rr], fma(sol_scale, w[i], xpre[rr][i]));
    }
  }
}

// Wide shape of the 3D Q4 FP32 colour pass (multiplicative, Boundary, and the first colour from
// zero): five patches per workgroup on 256 threads.  Its 49-line stages fill 245 of 256 lanes,
// against 98 of 128 for the two-patch default, which cuts the vector instructions per patch by
// about a fifth.  A row of patches along x0 that is not a multiple of five leaves a partial
// workgroup, so launches take it only on long rows (at most kWideIdle idle patch slots per row, as a
// fraction of the row).
#ifndef VPS_Q4_3D_WIDE
#define VPS_Q4_3D_WIDE 1
#endif
constexpr int kWidePPW = 5, kWideNT = 256;
constexpr double kWideIdle = 0.15;
template <int D, int K, typename T, int MODE>
struct HasWideForm {
  static constexpr bool value = D == 3 && K == 4 && sizeof(T) == 4 &&
                                (MODE == kModeMultiplicative || MODE == kModeZero || MODE == kModeBoundary) &&
                                VPS_Q4_3D_WIDE;
};
template <int D, int K, typename T, int MODE, int PPW>
struct IsWide {
  static constexpr bool value = HasWideForm<D, K, T, MODE>::value && PPW == kWidePPW;
};

// Degrees (bit K) whose default 3D multiplicative shape also takes the paired layout (the wide
// shape always does): 1-2.5% faster for degrees 5-7 (3D Q7: 30.8 -> 24.8 KB), equal for 3 and 4.
#ifndef VPS_3D_PAIR_MASK
#define VPS_3D_PAIR_MASK 0xE0
#endif
template <int D, int K, typename T, int MODE, int PPW>
struct LinesPair {
  static constexpr bool value =
      IsWide<D, K, T, MODE, PPW>::value ||
      (D == 3 && MODE == kModeMultiplicative && (((VPS_3D_PAIR_MASK) >> K) & 1) && PPW == SmootherShape<3, K>::PPW);
};

// Degrees (bit K) whose default 2D multiplicative shape takes the aliased LDS layout.
#ifndef VPS_2D_ALIAS_MASK
#define VPS_2D_ALIAS_MASK 0xFE
#endif

// The aliased LDS layout serves the default shape of the multiplicative pass where the shape asks
// for it, and the wide shape.
template <int D, int K, typename T, int MODE, int PPW>
struct LinesAlias {
  static constexpr bool value =
      (D == 3 && MODE == kModeMultiplicative && SmootherShape<3, K>::ALIAS && PPW == SmootherShape<3, K>::PPW) ||
      (D == 2 && MODE == kModeMultiplicative && (((VPS_2D_ALIAS_MASK) >> K) & 1) &&
       PPW == SmootherShape<2, K>::PPW) ||
      IsWide<D, K, T, MODE, PPW>::value;
};

// One workgroup's share of a colour pass: patches of block `blk` of the colour described by
// (p0, p1, p2, cnt0, cnt1, groups0) on a level with n1d nodes per direction.
template <int D, int K, typename T, int MODE, int PPW>
__device__ __forceinline__ void colour_pass_lines(T* __restrict__ smem, const T* __restrict__ b, T* __restrict__ x,
                                                  long long n1d, int p0, int p1, int p2, int cnt0, int cnt1,
                                                  int groups0, T res_scale, T sol_scale, unsigned blk) {
  constexpr int n = 2 * K + 1, m = 2 * K - 1, mm = m * m;
  constexpr int NT = IsWide<D, K, T, MODE, PPW>::value ? kWideNT : SmootherShape<D, K>::NT;
  // ZERO: the additive pass on x = 0 that also writes the zeros of the rest of its closures
  constexpr bool ZERO = MODE == kModeZero;
  constexpr bool ADD = MODE == kModeAdditive || ZERO, BND = MODE == kModeBoundary;
  // patch matrices and eigenvectors as compile-time constants (instruction literals / SGPR moves)
  using PT = gen::PatchTables<T, K>;
  using L = SmootherLds<D, K, T, ADD, PPW, LinesAlias<D, K, T, MODE, PPW>::value, LinesPair<D, K, T, MODE, PPW>::value>;
  constexpr int RS = L::RS;
  (void)p2;

  const ColourBlock cb = colour_block<D, K, PPW>(blk, p0, p1, p2, cnt0, cnt1, groups0);
  const int P = cb.count;
  const long long s0 = cb.s0, s1 = cb.s1, s2 = cb.s2;
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x;
  const int seg = 2 * K * P + 1;  // valid length of the closure row segment

  // Offsets inside one workgroup's block fit in 32 bits (checked by the launcher).
  const int ld1 = (int)n1d, ld2 = D == 3 ? (int)n1d2 : 0;
  const long long origin = (D == 3 ? s2 * n1d2 : 0) + s1 * n1d + s0;  // closure corner of the first patch
  T* xo = x + origin;  // same restrict object as x
  const T* bo = b + origin;

  // Lines along the slowest axis, task = (q, i1, i0) in 3D / (q, i0) in 2D with i0 fastest:
  // the residual stage reads b on them and the last stage updates x^I on them.  b is
  // prefetched now (clamped to a valid patch so the loads are always in bounds); the old x^I
  // comes from the closure in LDS in multiplicative mode and from global memory in additive mode.
  constexpr int NB = D == 3 ? PPW * mm : PPW * m;
  constexpr int RB = (NB + NT - 1) / NT;
  T bpre[RB][m], xpre[RB][m];
  unsigned loff[RB];  // byte offset of the line's first node from its plane
  int xoff[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    int q, i1 = 0, i0;
    if constexpr (D == 3) {
      q = task / mm;
      const int r = task - q * mm;
      i1 = r / m;
      i0 = r - i1 * m;
    } else {
      q = task / m;
      i0 = task - q * m;
    }
    q = min(q, P - 1);
    // node (1 + i1, 1 + i0) of the patch's first interior plane, relative to that plane
    const int off = (D == 3 ? (1 + i1) * ld1 : 0) + 2 * K * q + 1 + i0;
    loff[rr] = (unsigned)off * (unsigned)sizeof(T);
    xoff[rr] = (D == 3 ? (n + 1 + i1) * RS : RS) + 2 * K * q + 1 + i0;  // node (i=0) in the LDS closure
    const int st = D == 3 ? ld2 : ld1;
#pragma unroll
    for (int i = 0; i < m; ++i) bpre[rr][i] = ld_lane(bo + st + i * st, loff[rr]);
    if constexpr (ADD && !ZERO) {
#pragma unroll
      for (int i = 0; i < m; ++i) xpre[rr][i] = ld_lane(xo + st + i * st, loff[rr]);
    }
    if constexpr (ZERO) {
#pragma unroll
      for (int i = 0; i < m; ++i) xpre[rr][i] = T(0);
    }
  }

  if constexpr (ZERO) {
    // 0 on every closure node of the workgroup that is not a patch interior (neighbouring
    // workgroups write the same zeros on shared faces; no interior of the colour lies there).
    // Those nodes are the closure rows on its faces, whole, and on the other rows the columns
    // between patches (every 2k-th); rows run along x0.
    constexpr int NFR = D == 3 ? 4 * (n - 1) : 2;  // face rows (j2, j1) / (j1)
    constexpr int NIR = D == 3 ? m * m : m;        // other rows
    constexpr int NZF = NFR * RS, NZ = NZF + NIR * (PPW + 1);
    for (int w = tid; w < NZ; w += NT) {
      int j1, j2 = 0, c;
      if (w < NZF) {
        const int f = w / RS;
        c = w - f * RS;
        if constexpr (D == 3) {
          if (f < n) {
            j2 = 0;
            j1 = f;
          } else if (f < 2 * n) {
            j2 = n - 1;
            j1 = f - n;
          } else {
            j2 = 1 + (f - 2 * n) / 2;
            j1 = (f & 1) ? n - 1 : 0;  // f - 2n and f have the same parity (2n even)
          }
        } else {
          j1 = f == 0 ? 0 : n - 1;
        }
      } else {
        const int v = w - NZF, r = v / (PPW + 1);
        c = 2 * K * (v - r * (PPW + 1));
        if constexpr (D == 3) {
          j2 = 1 + r / m;
          j1 = 1 + (r - (r / m) * m);
        } else {
          j1 = 1 + r;
        }
      }
      if (c < seg) st_lane(xo, (unsigned)((D == 3 ? j2 * ld2 : 0) + j1 * ld1 + c) * (unsigned)sizeof(T), T(0));
    }
  }

  // ---- closure segment -> LDS X [j2][j1][c].  Work item = (column c, row j1 in 3D); the
  // slowest axis is walked unrolled.  Every closure node lies inside the grid: loads are
  // unconditional and Dirichlet nodes are replaced by 0 (boundary entries of x are ignored).
  // Boundary mode also replaces patch-interior nodes by 0 and does not load them: a column
  // strictly inside a patch along x0 (and x1 in 3D) needs only its two end nodes.
  if constexpr (!ADD) {
    T* X = smem + (D == 3 ? L::offX : L::offX2);
    constexpr int NW = D == 3 ? RS * n : RS;
    const bool lo1 = s1 == 0, hi1 = s1 + n - 1 == n1d - 1;
    const bool lo2 = D == 3 && s2 == 0, hi2 = D == 3 && s2 + n - 1 == n1d - 1;
    for (int w = tid; w < NW; w += NT) {
      const int c = w % RS, j1 = D == 3 ? w / RS : 0;
      const int cl = min(c, seg - 1);
      const long long gc = s0 + cl;
      bool bad = gc == 0 || gc == n1d - 1;
      if constexpr (D == 3) bad = bad || (j1 == 0 && lo1) || (j1 == n - 1 && hi1);
      const unsigned base = ((D == 3 ? j1 * ld1 : 0) + cl) * (unsigned)sizeof(T);
      const int sstride = D == 3 ? ld2 : ld1;
      // column strictly inside a patch (Boundary mode: its nodes 1..n-2 are patch-interior)
      const bool inner = BND && cl % (2 * K) != 0 && (D == 2 || (j1 > 0 && j1 < n - 1));
      T v[n];
#pragma unroll
      for (int j = 0; j < n; ++j) {
        if (BND && j > 0 && j < n - 1) {
          v[j] = inner ? T(0) : ld_lane(xo + j * sstride, base);
        } else {
          v[j] = ld_lane(xo + j * sstride, base);
        }
      }
      const bool lo = D == 3 ? lo2 : lo1, hi = D == 3 ? hi2 : hi1;
      if (c < seg) {
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const bool zero = bad || (j == 0 && lo) || (j == n - 1 && hi);
          X[(D == 3 ? j * n + j1 : j) * RS + c] = zero ? T(0) : v[j];
        }
      }
    }
    __syncthreads();
    if constexpr (!BND) {
      // old x^I of this thread's lines: patch-interior nodes are never Dirichlet nodes
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
#pragma unroll
        for (int i = 0; i < m; ++i) xpre[rr][i] = X[xoff[rr] + i * (D == 3 ? n * RS : RS)];
      }
    }
  }

  if constexpr (D == 3) {
    constexpr int SJ1 = L::SJ1, SJ2 = L::SJ2, SI1 = L::SI1, SI0 = L::SI0, SA1 = L::SA1, SA2 = L::SA2;
    if constexpr (!ADD) {
      const T* X = smem + L::offX;
      T* PM = smem + L::offP;  // [j1][q][j2][i0]
      T* PA = PM + n * SJ1;
      using T2 = typename Pair<T>::type;
      T2* PP = reinterpret_cast<T2*>(smem + L::offP);  // paired layout: [j1][q][j2][i0]{M, A}
      constexpr int SJP2 = L::SJP / 2;                  // pair stride
      // ---- contract x0 with Mc and Ac: lines (q, j2, j1), j1 fastest
      if constexpr (BND) {
        // Boundary form: the closure is zero on patch-interior nodes, so an x0 line with j2 and j1
        // both interior holds only its two end values.  The 4(n-1) face lines of each patch come
        // first and take the full contraction, the m^2 interior lines a two-term one.
        constexpr int NF = 4 * (n - 1);
        // face tasks padded to whole waves, so that no wave mixes the two kinds of line
        constexpr int FP = (PPW * NF + 63) / 64 * 64, NTASK = FP + PPW * mm;
        // task -> line (q, j2, j1); false for padding and for patches past the workgroup's last
        auto line_of = [&](int task, int& q, int& j2, int& j1) -> bool {
          if (task >= NTASK || (task >= PPW * NF && task < FP)) return false;
          if (task < FP) {
            q = task / NF;
            const int f = task - q * NF;
            if (f < n) {
              j2 = 0;
              j1 = f;
            } else if (f < 2 * n) {
              j2 = n - 1;
              j1 = f - n;
            } else {
              j2 = 1 + (f - 2 * n) / 2;
              j1 = (f & 1) ? n - 1 : 0;  // f - 2n and f have the same parity (2n even)
            }
          } else {
            const int t = task - FP;
            q = t / mm;
            const int c = t - q * mm;
            j2 = 1 + c / m;
            j1 = 1 + (c - (c / m) * m);
          }
          return q < P;
        };
        // M and A rows of one line into sm, sa
        auto contract = [&](bool face, int row, T* sm, T* sa) {
          if (face) {
            T in[n];
#pragma unroll
            for (int j = 0; j < n; ++j) in[j] = X[row + j];
#pragma unroll
            for (int i = 0; i < m; ++i) {
              T am = T(0), aa = T(0);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                am = fma_tab(PT::Mc[i * n + j], in[j], am);
                aa = fma_tab(PT::Ac[i * n + j], in[j], aa);
              }
              sm[i] = am;
              sa[i] = aa;
            }
          } else {
            const T e0 = X[row], e1 = X[row + n - 1];
#pragma unroll
            for (int i = 0; i < m; ++i) {
              sm[i] = fma_tab(PT::Mc[i * n], e0, fma_tab(PT::Mc[i * n + n - 1], e1, T(0)));
              sa[i] = fma_tab(PT::Ac[i * n], e0, fma_tab(PT::Ac[i * n + n - 1], e1, T(0)));
            }
          }
        };
        if constexpr (L::AL) {
          // aliased: every line is read and contracted, then PM/PA overwrite X
          constexpr int RA = (NTASK + NT - 1) / NT;
          T om[RA][m], oa[RA][m];
#pragma unroll
          for (int rr = 0; rr < RA; ++rr) {
            const int task = rr * NT + tid;
            int q, j2, j1;
            if (line_of(task, q, j2, j1))
              contract(task < FP, lds_base((j2 * n + j1) * RS + 2 * K * q), om[rr], oa[rr]);
          }
          __syncthreads();
#pragma unroll
          for (int rr = 0; rr < RA; ++rr) {
            const int task = rr * NT + tid;
            int q, j2, j1;
            if (line_of(task, q, j2, j1)) {
              if constexpr (L::PR) {
                const int o = lds_base(j1 * SJP2 + (q * n + j2) * m);
#pragma unroll
                for (int i = 0; i < m; ++i) PP[o + i] = T2{om[rr][i], oa[rr][i]};
              } else {
                const int o = lds_base(j1 * SJ1 + (q * n + j2) * m);
#pragma unroll
                for (int i = 0; i < m; ++i) {
                  PM[o + i] = om[rr][i];
                  PA[o + i] = oa[rr][i];
                }
              }
            }
          }
        } else {
          for (int base = 0; base < NTASK; base += NT) {
            const int task = base + tid;
            int q, j2, j1;
            if (!line_of(task, q, j2, j1)) continue;
            const int o = lds_base(j1 * SJ1 + (q * n + j2) * m);
            T sm[m], sa[m];
            contract(task < FP, lds_base((j2 * n + j1) * RS + 2 * K * q), sm, sa);
#pragma unroll
            for (int i = 0; i < m; ++i) {
              PM[o + i] = sm[i];
              PA[o + i] = sa[i];
            }
          }
        }
      } else if constexpr (L::AL) {
        // aliased: every line of the workgroup is read and contracted, then PM/PA overwrite X
        constexpr int NA = PPW * n * n, RA = (NA + NT - 1) / NT;
        T om[RA][m], oa[RA][m];
#pragma unroll
        for (int rr = 0; rr < RA; ++rr) {
          const int task = rr * NT + tid;
          const int q = task / (n * n), r = task - q * (n * n);
          const int j2 = r / n, j1 = r - j2 * n;
          if (task < NA && q < P) {
            T in[n];
            const int row = lds_base((j2 * n + j1) * RS + 2 * K * q);
#pragma unroll
            for (int j = 0; j < n; ++j) in[j] = X[row + j];
#pragma unroll
            for (int i = 0; i < m; ++i) {
              T sm = T(0), sa = T(0);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                sm = fma_tab(PT::Mc[i * n + j], in[j], sm);
                sa = fma_tab(PT::Ac[i * n + j], in[j], sa);
              }
              om[rr][i] = sm;
              oa[rr][i] = sa;
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < RA; ++rr) {
          const int task = rr * NT + tid;
          const int q = task / (n * n), r = task - q * (n * n);
          const int j2 = r / n, j1 = r - j2 * n;
          if (task < NA && q < P) {
            if constexpr (L::PR) {
              const int o = lds_base(j1 * SJP2 + (q * n + j2) * m);
#pragma unroll
              for (int i = 0; i < m; ++i) PP[o + i] = T2{om[rr][i], oa[rr][i]};
            } else {
              const int o = lds_base(j1 * SJ1 + (q * n + j2) * m);
#pragma unroll
              for (int i = 0; i < m; ++i) {
                PM[o + i] = om[rr][i];
                PA[o + i] = oa[rr][i];
              }
            }
          }
        }
      } else
      for (int base = 0; base < PPW * n * n; base += NT) {
        const int task = base + tid;
        const int q = task / (n * n), r = task - q * (n * n);
        const int j2 = r / n, j1 = r - j2 * n;
        if (task < PPW * n * n && q < P) {
          T in[n];
          const int row = lds_base((j2 * n + j1) * RS + 2 * K * q);
#pragma unroll
          for (int j = 0; j < n; ++j) in[j] = X[row + j];
          const int o = lds_base(j1 * SJ1 + (q * n + j2) * m);
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sm = fma_tab(PT::Mc[i * n + j], in[j], sm);
            PM[o + i] = sm;
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sa = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sa = fma_tab(PT::Ac[i * n + j], in[j], sa);
            PA[o + i] = sa;
          }
        }
      }
      __syncthreads();
      // ---- contract x1: lines (q, j2, i0), i0 fastest; U = M1 (M0 x), V = A1 (M0 x) + M1 (A0 x)
      T* U = smem + L::offUV;  // [j2][q][i1][i0]
      T* V = U + n * SJ2;
      if constexpr (L::AL) {
        // aliased: U/V overwrite PM/PA once every line has been read
        constexpr int NB2 = PPW * n * m, RB2 = (NB2 + NT - 1) / NT;
        T ou[RB2][m], ov[RB2][m];
#pragma unroll
        for (int rr = 0; rr < RB2; ++rr) {
          const int task = rr * NT + tid;
          const int q = task / (n * m);
          if (task < NB2 && q < P) {
            T pm[n], pa[n];
#pragma unroll
            for (int j = 0; j < n; ++j) {
              if constexpr (L::PR) {
                const T2 v = PP[j * SJP2 + task];
                pm[j] = v.x;
                pa[j] = v.y;
              } else {
                pm[j] = PM[j * SJ1 + task];
                pa[j] = PA[j * SJ1 + task];
              }
            }
#pragma unroll
            for (int i = 0; i < m; ++i) {
              T su = T(0), sv = T(0);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                su = fma_tab(PT::Mc[i * n + j], pm[j], su);
                sv = fma_tab(PT::Ac[i * n + j], pm[j], sv);
                sv = fma_tab(PT::Mc[i * n + j], pa[j], sv);
              }
              ou[rr][i] = su;
              ov[rr][i] = sv;
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < RB2; ++rr) {
          const int task = rr * NT + tid;
          const int q = task / (n * m), r = task - q * (n * m);
          const int j2 = r / m, i0 = r - j2 * m;
          if (task < NB2 && q < P) {
            const int o = lds_base(j2 * SJ2 + q * mm + i0);
#pragma unroll
            for (int i = 0; i < m; ++i) {
              U[o + i * m] = ou[rr][i];
              V[o + i * m] = ov[rr][i];
            }
          }
        }
      } else
      for (int base = 0; base < PPW * n * m; base += NT) {
        const int task = base + tid;
        const int q = task / (n * m), r = task - q * (n * m);
        const int j2 = r / m, i0 = r - j2 * m;
        if (task < PPW * n * m && q < P) {
          T pm[n], pa[n];
          const int ri = task;  // = (q * n + j2) * m + i0
#pragma unroll
          for (int j = 0; j < n; ++j) {
            pm[j] = PM[j * SJ1 + ri];
            pa[j] = PA[j * SJ1 + ri];
          }
          const int o = lds_base(j2 * SJ2 + q * mm + i0);
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T su = T(0), sv = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              su = fma_tab(PT::Mc[i * n + j], pm[j], su);
              sv = fma_tab(PT::Ac[i * n + j], pm[j], sv);
              sv = fma_tab(PT::Mc[i * n + j], pa[j], sv);
            }
            U[o + i * m] = su;
            V[o + i * m] = sv;
          }
        }
      }
      __syncthreads();
    }
    // ---- contract x2 (residual) and apply Sᵀ along x2: lines (q, i1, i0), i0 fastest.  Paired
    // layout: W4 overwrites U/V, so every line is computed before the workgroup synchronises and
    // writes.
    T* W4 = smem + L::offW46;  // [i1][q][a2][i0]
    T tc[RB][m];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / mm, r = task - q * mm;
      const int i1 = r / m, i0 = r - i1 * m;
      if (task < NB && q < P) {
        T res[m];
        if constexpr (ADD) {
#pragma unroll
          for (int i = 0; i < m; ++i) res[i] = bpre[rr][i];
        } else {
          const T* U = smem + L::offUV;
          const T* V = U + n * SJ2;
          T u[n], v[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            u[j] = U[j * SJ2 + task];
            v[j] = V[j * SJ2 + task];
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              s = fma_tab(PT::Ac[i * n + j], u[j], s);
              s = fma_tab(PT::Mc[i * n + j], v[j], s);
            }
            res[i] = fma(-res_scale, s, bpre[rr][i]);
          }
        }
        apply_st<T, K>(res, tc[rr]);
        if constexpr (!L::PR) {
          const int o = lds_base(i1 * SI1 + q * mm + i0);
#pragma unroll
          for (int a = 0; a < m; ++a) W4[o + a * m] = tc[rr][a];
        }
      }
    }
    if constexpr (L::PR) {
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int task = rr * NT + tid;
        const int q = task / mm, r = task - q * mm;
        const int i1 = r / m, i0 = r - i1 * m;
        if (task < NB && q < P) {
          const int o = lds_base(i1 * SI1 + q * mm + i0);
#pragma unroll
          for (int a = 0; a < m; ++a) W4[o + a * m] = tc[rr][a];
        }
      }
    }
    __syncthreads();
    // ---- Sᵀ along x1: lines (q, a2, i0), i0 fastest
    T* W5 = smem + L::offW57;  // [i0][q][a2][a1]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        T in[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W4[i * SI1 + task];
        const int o = lds_base(i0 * SI0 + q * mm + a2 * m);
        T t[m];
        apply_st<T, K>(in, t);
#pragma unroll
        for (int a = 0; a < m; ++a) W5[o + a] = t[a];
      }
    }
    __syncthreads();
    // ---- Sᵀ along x0, scale by 1/(lam2+lam1+lam0), S along x0: lines (q, a2, a1), a1 fastest
    T* W6 = smem + L::offW46;  // [a1][q][a2][i0]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, a1 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m], z[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W5[i * SI0 + task];
        const int li = (a2 * m + a1) * m;
        apply_st<T, K>(in, z);
#pragma unroll
        for (int a = 0; a < m; ++a) z[a] *= tb.inv3[li + a];
        const int o = lds_base(a1 * SA1 + q * mm + a2 * m);
        T w[m];
        apply_s<T, K>(z, w);
#pragma unroll
        for (int i = 0; i < m; ++i) W6[o + i] = w[i];
      }
    }
    __syncthreads();
    // ---- S along x1: lines (q, a2, i0), i0 fastest
    T* W7 = smem + L::offW57;  // [a2][q][i1][i0]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W6[a * SA1 + task];
        const int o = lds_base(a2 * SA2 + q * mm + i0);
        T w[m];
        apply_s<T, K>(in, w);
#pragma unroll
        for (int i = 0; i < m; ++i) W7[o + i * m] = w[i];
      }
    }
    __syncthreads();
    // ---- S along x2 and x^I += correction, straight to global: lines (q, i1, i0)
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / mm;
      if (task < NB && q < P) {
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W7[a * SA2 + task];
        T w[m];
        apply_s<T, K>(in, w);
#pragma unroll
        for (int i = 0; i < m; ++i)
          st_lane(xo + (1 + i) * ld2, loff[rr], BND ? sol_scale * w[i] : fma(sol_scale, w[i], xpre[rr][i]));
      }
    }
  } else {
    // ================================ 2D =====================================
    constexpr int T1 = L::T1, T0 = L::T0, TA = L::TA;
    if constexpr (!ADD) {
      const T* X = smem + L::offX2;
      T* PM = smem + L::offP2;  // [j1][q][i0]
      T* PA = PM + n * T1;
      // ---- contract x0 with Mc and Ac: lines (q, j1), q fastest
      if constexpr (L::AL2) {
        // aliased: every line is read and contracted, then PM/PA overwrite X
        constexpr int R0 = (PPW * n + NT - 1) / NT;
        T om[R0][m], oa[R0][m];
#pragma unroll
        for (int rr = 0; rr < R0; ++rr) {
          const int task = rr * NT + tid;
          const int j1 = task / PPW, q = task - j1 * PPW;
          if (task < PPW * n && q < P) {
            T in[n];
#pragma unroll
            for (int j = 0; j < n; ++j) in[j] = X[j1 * RS + 2 * K * q + j];
#pragma unroll
            for (int i = 0; i < m; ++i) {
              T sm = T(0), sa = T(0);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                sm = fma_tab(PT::Mc[i * n + j], in[j], sm);
                sa = fma_tab(PT::Ac[i * n + j], in[j], sa);
              }
              om[rr][i] = sm;
              oa[rr][i] = sa;
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < R0; ++rr) {
          const int task = rr * NT + tid;
          const int j1 = task / PPW, q = task - j1 * PPW;
          if (task < PPW * n && q < P) {
            const int o = lds_base(j1 * T1 + q * m);
#pragma unroll
            for (int i = 0; i < m; ++i) {
              PM[o + i] = om[rr][i];
              PA[o + i] = oa[rr][i];
            }
          }
        }
      } else
      for (int base = 0; base < PPW * n; base += NT) {
        const int task = base + tid;
        const int j1 = task / PPW, q = task - j1 * PPW;
        if (task < PPW * n && q < P) {
          T in[n];
#pragma unroll
          for (int j = 0; j < n; ++j) in[j] = X[j1 * RS + 2 * K * q + j];
          const int o = lds_base(j1 * T1 + q * m);
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sm = fma_tab(PT::Mc[i * n + j], in[j], sm);
            PM[o + i] = sm;
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T sa = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) sa = fma_tab(PT::Ac[i * n + j], in[j], sa);
            PA[o + i] = sa;
          }
        }
      }
      __syncthreads();
    }
    // ---- residual along x1, r = b - (A1 (M0 x) + M1 (A0 x)) (or r = b), then Sᵀ along x1:
    //      lines (q, i0), i0 fastest.  Aliased layout: W overwrites PM/PA, so every line is
    //      computed before the workgroup synchronises and writes.
    T* W = smem + L::offW;  // [i0][q][a1]
    T tw[RB][m];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / m;
      if (task < NB && q < P) {
        T res[m];
        if constexpr (ADD) {
#pragma unroll
          for (int i = 0; i < m; ++i) res[i] = bpre[rr][i];
        } else {
          const T* PM = smem + L::offP2;
          const T* PA = PM + n * T1;
          T pm[n], pa[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            pm[j] = PM[j * T1 + task];
            pa[j] = PA[j * T1 + task];
          }
#pragma unroll
          for (int i = 0; i < m; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              s = fma_tab(PT::Ac[i * n + j], pm[j], s);
              s = fma_tab(PT::Mc[i * n + j], pa[j], s);
            }
            res[i] = fma(-res_scale, s, bpre[rr][i]);
          }
        }
        apply_st<T, K>(res, tw[rr]);
      }
    }
    if constexpr (L::AL2) __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / m, i0 = task - q * m;
      if (task < NB && q < P) {
        const int o = lds_base(i0 * T0 + q * m);
#pragma unroll
        for (int a = 0; a < m; ++a) W[o + a] = tw[rr][a];
      }
    }
    __syncthreads();
    // ---- Sᵀ along x0, scale by 1/(lam1+lam0), S along x0: lines (q, a1), a1 fastest
    T* W2 = smem + L::offW2;  // [a1][q][i0]
    for (int base = 0; base < PPW * m; base += NT) {
      const int task = base + tid;
      const int q = task / m, a1 = task - q * m;
      if (task < PPW * m && q < P) {
        const DevTables<T>& tb = tab_fresh<T>(K);
        T in[m], z[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W[i * T0 + task];
        apply_st<T, K>(in, z);
#pragma unroll
        for (int a = 0; a < m; ++a) z[a] *= tb.inv2[a1 * m + a];
        const int o = lds_base(a1 * TA + q * m);
        T w[m];
        apply_s<T, K>(z, w);
#pragma unroll
        for (int i = 0; i < m; ++i) W2[o + i] = w[i];
      }
    }
    __syncthreads();
    // ---- S along x1 and x^I += correction, straight to global: lines (q, i0)
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / m;
      if (task < NB && q < P) {
        T in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W2[a * TA + task];
        T w[m];
        apply_s<T, K>(in, w);
#pragma unroll
        for (int i = 0; i < m; ++i)
          st_lane(xo + (1 + i) * ld1, loff[rr], BND ? sol_scale * w[i] : fma(sol_scale, w[i], xpre[rr][i]));
      }
    }
  }
}

// ------------------------------------------------------------------ matrix-core form (3D, FP32)
//
// The three contractions of the localised residual r = b - Abar x (Sec. 3.1.1) are dense products
// of a batch of patch lines with one small 1D matrix, so they run on the matrix cores
// (v_mfma_f32_16x16x4f32: 16 lines x 4 inputs times 4 inputs x 16 outputs, FP32 products
// accumulated in FP32); the fast-diagonalisation stages stay on the vector ALU, where the
// eigenvectors' mirror symmetry halves their multiply-adds.  Lines of the workgroup's PPW
// patches are stacked into 16-row tiles; the 1D matrices sit in per-lane registers (B operand):
//   x0: lines (q, j2, j1) of the closure, inputs c (n, padded to a multiple of 4), outputs
//       [M0 x | A0 x] (2m <= 16)                                  -> PM, PA [i0][line]
//   x1: lines (q, i0, j2), inputs [PM(j1) | PA(j1)] (2n), outputs
//       [M1 PM | A1 PM + M1 PA] (2m)                               -> U, V  [i1][line]
//   x2: lines (q, i1, i0), inputs [U(j2) | V(j2)] (2n), outputs A2 U + M2 V (m); the vector ALU
//       then forms r = b - h (A2 U + M2 V) and applies S^T along x2, as in colour_pass_lines.
// Matrix-core operand layout (16x16x4, FP32): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[4 (l / 16) + i][l % 16] in accumulator register i.
template <int K, int PPW>
struct MfmaLds {
  static constexpr int n = 2 * K + 1, m = 2 * K - 1, mm = m * m, nn = n * n;
  static constexpr int KB0 = (n + 3) / 4, KB1 = (2 * n + 3) / 4;     // 4-wide input blocks
  static constexpr int R0 = PPW * nn, R1 = PPW * m * n, R2 = PPW * mm;  // lines per stage
  static constexpr int T0 = (R0 + 15) / 16, T1 = (R1 + 15) / 16, T2 = (R2 + 15) / 16;
  static constexpr int RS = 2 * K * PPW + 1;
  // closure rows padded so that a tile's 4-wide input blocks past column n stay inside the row (their
  // B rows are zero; the values read there are zeros written by the closure load), and = 4 (mod 32)
  // so that the 16 rows of a tile fall into distinct bank groups
  static constexpr int RSX = pad32(RS + 4 * KB0 - n, 4);
  static constexpr int LS0 = pad32(16 * T0, 20);   // PM / PA row: tile writes of 4 lines at once
  static constexpr int LS1 = pad32(16 * T1, 4);    // U / V row
  static constexpr int LS2 = pad32(16 * T2, 4);    // x2 result row
  static constexpr int X = nn * RSX;
  static constexpr int P = 2 * m * LS0;            // PM, PA
  static constexpr int UV = 2 * m * LS1;           // U, V
  static constexpr int Q = m * LS2;                // A2 U + M2 V
  using Fd = SmootherLds<3, K, float, false, PPW>;  // strides of the diagonalisation stages
  static constexpr int FD = m * (Fd::SI1 > Fd::SI0 ? (Fd::SI1 > Fd::SA1 ? (Fd::SI1 > Fd::SA2 ? Fd::SI1 : Fd::SA2)
                                                                         : (Fd::SA1 > Fd::SA2 ? Fd::SA1 : Fd::SA2))
                                                   : (Fd::SI0 > Fd::SA1 ? (Fd::SI0 > Fd::SA2 ? Fd::SI0 : Fd::SA2)
                                                                         : (Fd::SA1 > Fd::SA2 ? Fd::SA1 : Fd::SA2)));
  static constexpr int max2(int a, int b) { return a > b ? a : b; }
  // region 0: X, then U/V, then the diagonalisation buffers of odd stages; region 1: PM/PA, then Q,
  // then the even ones
  static constexpr int A = max2(max2(X, UV), FD);
  static constexpr int B = max2(max2(P, Q), FD);
  static constexpr int total = A + B;
};

typedef float vps_f32x4 __attribute__((ext_vector_type(4)));

template <int K, int PPW>
__device__ __forceinline__ void colour_pass_mfma3(float* __restrict__ smem, const float* __restrict__ b,
                                                  float* __restrict__ x, long long n1d, int p0, int p1, int p2,
                                                  int cnt0, int cnt1, int groups0, float res_scale, float sol_scale,
                                                  unsigned blk) {
  using L = MfmaLds<K, PPW>;
  using PT = gen::PatchTables<float, K>;
  using Fd = typename L::Fd;
  constexpr int n = L::n, m = L::m, mm = L::mm, nn = L::nn, RS = L::RS, RSX = L::RSX;
  constexpr int NT = 256, NW = NT / 64;
  static_assert(2 * m <= 16, "outputs of one contraction must fit the 16 matrix columns");
  float* const rA = smem;         // X, then U/V, then odd diagonalisation buffers
  float* const rB = smem + L::A;  // PM/PA, then Q, then even ones

  const ColourBlock cb = colour_block<3, K, PPW>(blk, p0, p1, p2, cnt0, cnt1, groups0);
  const int P = cb.count;
  const long long s0 = cb.s0, s1 = cb.s1, s2 = cb.s2;
  const long long n1d2 = n1d * n1d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;  // matrix-core row (A) / column (B, D) and input sub-index
  const int seg = 2 * K * P + 1;             // valid closure columns along x0
  const int ld1 = (int)n1d, ld2 = (int)n1d2;
  float* xo = x + (s2 * n1d2 + s1 * n1d + s0);
  const float* bo = b + (s2 * n1d2 + s1 * n1d + s0);

  // B operands (1D patch matrices; zero rows pad the inputs, zero columns the outputs)
  float bx0[L::KB0], bx1[L::KB1], bx2[L::KB1];
#pragma unroll
  for (int kb = 0; kb < L::KB0; ++kb) {
    const int k = 4 * kb + lk;
    bx0[kb] = k >= n ? 0.f : lr < m ? PT::Mc[lr * n + k] : lr < 2 * m ? PT::Ac[(lr - m) * n + k] : 0.f;
  }
#pragma unroll
  for (int kb = 0; kb < L::KB1; ++kb) {
    const int k = 4 * kb + lk;
    const bool pm = k < n, pa = k >= n && k < 2 * n;
    const int c = pm ? k : k - n;
    bx1[kb] = lr < m ? (pm ? PT::Mc[lr * n + c] : 0.f)
                     : lr < 2 * m ? (pm ? PT::Ac[(lr - m) * n + c] : pa ? PT::Mc[(lr - m) * n + c] : 0.f) : 0.f;
    bx2[kb] = lr < m ? (pm ? PT::Ac[lr * n + c] : pa ? PT::Mc[lr * n + c] : 0.f) : 0.f;
  }

  // Lines (q, i1, i0) of the vector stages: b on them is prefetched now (tasks past the last patch
  // are clamped to it, so every load is in bounds)
  constexpr int NB = PPW * mm;
  constexpr int RB = (NB + NT - 1) / NT;
  float bpre[RB][m], xpre[RB][m];
  unsigned loff[RB];
  int xoff[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int task = rr * NT + tid;
    int q = task / mm;
    const int r = task - q * mm, i1 = r / m, i0 = r - i1 * m;
    q = min(q, P - 1);
    loff[rr] = (unsigned)((1 + i1) * ld1 + 2 * K * q + 1 + i0) * (unsigned)sizeof(float);
    xoff[rr] = (n + 1 + i1) * RSX + 2 * K * q + 1 + i0;  // node (i = 0) in the LDS closure
#pragma unroll
    for (int i = 0; i < m; ++i) bpre[rr][i] = ld_lane(bo + ld2 + i * ld2, loff[rr]);
  }

  // ---- closure -> X [j2][j1][c]; Dirichlet nodes, and columns past the workgroup's last patch, are 0
  {
    float* X = rA;
    const bool lo1 = s1 == 0, hi1 = s1 + n - 1 == n1d - 1;
    const bool lo2 = s2 == 0, hi2 = s2 + n - 1 == n1d - 1;
    for (int w = tid; w < RSX * n; w += NT) {
      const int j1 = w / RSX, c = w - j1 * RSX;
      const int cl = min(c, seg - 1);
      const long long gc = s0 + cl;
      const bool bad = c >= seg || gc == 0 || gc == n1d - 1 || (j1 == 0 && lo1) || (j1 == n - 1 && hi1);
      const unsigned base = (unsigned)(j1 * ld1 + cl) * (unsigned)sizeof(float);
      float v[n];
#pragma unroll
      for (int j = 0; j < n; ++j) v[j] = ld_lane(xo + j * ld2, base);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const bool zero = bad || (j == 0 && lo2) || (j == n - 1 && hi2);
        X[(j * n + j1) * RSX + c] = zero ? 0.f : v[j];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
#pragma unroll
    for (int i = 0; i < m; ++i) xpre[rr][i] = rA[xoff[rr] + i * n * RSX];  // old x^I (never Dirichlet)
  }

  // ---- x0 on the matrix cores: lines (q, j2, j1) -> PM, PA [i0][line]
  {
    const float* X = rA;
    float* PM = rB;
    for (int t = wave; t < L::T0; t += NW) {
      const int row = min(16 * t + lr, L::R0 - 1);
      const int q = row / nn, rem = row - q * nn;
      const int a = lds_base(rem * RSX + 2 * K * q + lk);
      vps_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < L::KB0; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[a + 4 * kb], bx0[kb], acc, 0, 0, 0);
      if (lr < 2 * m) *reinterpret_cast<vps_f32x4*>(PM + lr * L::LS0 + 16 * t + 4 * lk) = acc;
    }
  }
  __syncthreads();
  // ---- x1 on the matrix cores: lines (q, i0, j2), inputs PM(j1), PA(j1) -> U, V [i1][line]
  {
    const float* PM = rB;
    float* U = rA;
    int koff[L::KB1];
#pragma unroll
    for (int kb = 0; kb < L::KB1; ++kb) {
      const int k = 4 * kb + lk;
      koff[kb] = k < n ? k : k < 2 * n ? m * L::LS0 + (k - n) : 0;
    }
    for (int t = wave; t < L::T1; t += NW) {
      const int row = min(16 * t + lr, L::R1 - 1);
      const int q = row / (m * n), rem = row - q * (m * n);
      const int i0 = rem / n, j2 = rem - i0 * n;
      const int a = lds_base(i0 * L::LS0 + q * nn + j2 * n);
      vps_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < L::KB1; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(PM[a + koff[kb]], bx1[kb], acc, 0, 0, 0);
      if (lr < 2 * m) *reinterpret_cast<vps_f32x4*>(U + lr * L::LS1 + 16 * t + 4 * lk) = acc;
    }
  }
  __syncthreads();
  // ---- x2 on the matrix cores: lines (q, i1, i0), inputs U(j2), V(j2) -> Q = A2 U + M2 V [i2][line]
  {
    const float* U = rA;
    float* Q = rB;
    int koff[L::KB1];
#pragma unroll
    for (int kb = 0; kb < L::KB1; ++kb) {
      const int k = 4 * kb + lk;
      koff[kb] = k < n ? k : k < 2 * n ? m * L::LS1 + (k - n) : 0;
    }
    for (int t = wave; t < L::T2; t += NW) {
      const int row = min(16 * t + lr, L::R2 - 1);
      const int q = row / mm, rem = row - q * mm;
      const int i1 = rem / m, i0 = rem - i1 * m;
      const int a = lds_base(i1 * L::LS1 + (q * m + i0) * n);
      vps_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < L::KB1; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(U[a + koff[kb]], bx2[kb], acc, 0, 0, 0);
      if (lr < m) *reinterpret_cast<vps_f32x4*>(Q + lr * L::LS2 + 16 * t + 4 * lk) = acc;
    }
  }
  __syncthreads();

  constexpr int SI1 = Fd::SI1, SI0 = Fd::SI0, SA1 = Fd::SA1, SA2 = Fd::SA2;
  // ---- r = b - h (A2 U + M2 V), then S^T along x2: lines (q, i1, i0)
  {
    const float* Q = rB;
    float* W4 = rA;  // [i1][q][a2][i0]
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / mm, r = task - q * mm;
      const int i1 = r / m, i0 = r - i1 * m;
      if (task < NB && q < P) {
        float res[m];
#pragma unroll
        for (int i = 0; i < m; ++i) res[i] = fma(-res_scale, Q[i * L::LS2 + task], bpre[rr][i]);
        float t[m];
        apply_st<float, K>(res, t);
        const int o = lds_base(i1 * SI1 + q * mm + i0);
#pragma unroll
        for (int a = 0; a < m; ++a) W4[o + a * m] = t[a];
      }
    }
  }
  __syncthreads();
  // ---- S^T along x1: lines (q, a2, i0)
  {
    const float* W4 = rA;
    float* W5 = rB;  // [i0][q][a2][a1]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        float in[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W4[i * SI1 + task];
        const int o = lds_base(i0 * SI0 + q * mm + a2 * m);
        float t[m];
        apply_st<float, K>(in, t);
#pragma unroll
        for (int a = 0; a < m; ++a) W5[o + a] = t[a];
      }
    }
  }
  __syncthreads();
  // ---- S^T along x0, 1/(lam2 + lam1 + lam0), S along x0: lines (q, a2, a1)
  {
    const float* W5 = rB;
    float* W6 = rA;  // [a1][q][a2][i0]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, a1 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        const DevTables<float>& tb = tab_fresh<float>(K);
        float in[m], z[m];
#pragma unroll
        for (int i = 0; i < m; ++i) in[i] = W5[i * SI0 + task];
        const int li = (a2 * m + a1) * m;
        apply_st<float, K>(in, z);
#pragma unroll
        for (int a = 0; a < m; ++a) z[a] *= tb.inv3[li + a];
        const int o = lds_base(a1 * SA1 + q * mm + a2 * m);
        float w[m];
        apply_s<float, K>(z, w);
#pragma unroll
        for (int i = 0; i < m; ++i) W6[o + i] = w[i];
      }
    }
  }
  __syncthreads();
  // ---- S along x1: lines (q, a2, i0)
  {
    const float* W6 = rA;
    float* W7 = rB;  // [a2][q][i1][i0]
    for (int base = 0; base < PPW * mm; base += NT) {
      const int task = base + tid;
      const int q = task / mm, r = task - q * mm;
      const int a2 = r / m, i0 = r - a2 * m;
      if (task < PPW * mm && q < P) {
        float in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W6[a * SA1 + task];
        const int o = lds_base(a2 * SA2 + q * mm + i0);
        float w[m];
        apply_s<float, K>(in, w);
#pragma unroll
        for (int i = 0; i < m; ++i) W7[o + i * m] = w[i];
      }
    }
  }
  __syncthreads();
  // ---- S along x2 and x^I += correction / h, straight to global: lines (q, i1, i0)
  {
    const float* W7 = rB;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int task = rr * NT + tid;
      const int q = task / mm;
      if (task < NB && q < P) {
        float in[m];
#pragma unroll
        for (int a = 0; a < m; ++a) in[a] = W7[a * SA2 + task];
        float w[m];
        apply_s<float, K>(in, w);
#pragma unroll
        for (int i = 0; i < m; ++i) st_lane(xo + (1 + i) * ld2, loff[rr], fma(sol_scale, w[i], xpre[rr][i]));
      }
    }
  }
}

// LDS words of one workgroup of a colour pass.  The x2-first form (colour_pass_mult3) serves the 3D
// multiplicative pass in FP64, where it measured 3-9% faster than the closure-through-LDS form; in
// FP32 the two measured within 2% and the closure form is kept (its b loads stay within one node
// plane per access).
// Patches per workgroup of the matrix-core form (3D Q4, FP32, multiplicative), 256 threads.
constexpr int kMfmaPPW = 4;
template <int D, int K, typename T>
struct HasMfmaForm {
  static constexpr bool value = D == 3 && K == 4 && sizeof(T) == 4;
};
template <int D, int K, typename T, int MODE>
struct UsesMfma {
  static constexpr bool value = HasMfmaForm<D, K, T>::value && MODE == kModeMfma;
};
// Default launch shape per form: patches per workgroup and threads.
template <int D, int K, typename T, int MODE>
struct ColourShape {
  static constexpr bool kMfma = UsesMfma<D, K, T, MODE>::value;
  static constexpr int PPW = kMfma ? kMfmaPPW : SmootherShape<D, K>::PPW;
  static constexpr int NT = kMfma ? 256 : SmootherShape<D, K>::NT;
};
// Threads of a launch with PPW patches per workgroup (small launches take the vector form with the
// latency shape).
template <int D, int K, typename T, int MODE, int PPW>
struct ColourNT {
  static constexpr int value = UsesMfma<D, K, T, MODE>::value && PPW == kMfmaPPW ? 256
                               : IsWide<D, K, T, MODE, PPW>::value               ? kWideNT
                                                                                 : SmootherShape<D, K>::NT;
};

template <int D, int K, typename T, int MODE, int PPW>
struct ColourLds {
  static constexpr bool kMfma = UsesMfma<D, K, T, MODE>::value && PPW == kMfmaPPW;
  static constexpr bool kMult3 = D == 3 && MODE == kModeMultiplicative && sizeof(T) == 8;
  static constexpr int value = kMfma ? MfmaLds<K, PPW>::total
                               : kMult3 ? Mult3Lds<K, PPW>::total
                                        : SmootherLds<D, K, T, MODE == kModeAdditive || MODE == kModeZero, PPW,
                                                      LinesAlias<D, K, T, MODE, PPW>::value,
                                                      LinesPair<D, K, T, MODE, PPW>::value>::total;
};

// One workgroup's share of a colour pass: the 3D multiplicative pass in FP64 contracts the closure
// along x2 first; the other forms run the closure through LDS (colour_pass_lines).
template <int D, int K, typename T, int MODE, int PPW>
__device__ __forceinline__ void colour_pass_block(T* __restrict__ smem, const T* __restrict__ b, T* __restrict__ x,
                                                  long long n1d, int p0, int p1, int p2, int cnt0, int cnt1,
                                                  int groups0, T res_scale, T sol_scale, unsigned blk) {
  if constexpr (ColourLds<D, K, T, MODE, PPW>::kMfma)
    colour_pass_mfma3<K, PPW>(smem, b, x, n1d, p0, p1, p2, cnt0, cnt1, groups0, res_scale, sol_scale, blk);
  else if constexpr (ColourLds<D, K, T, MODE, PPW>::kMult3)
    colour_pass_mult3<K, T, PPW>(smem, b, x, n1d, p0, p1, p2, cnt0, cnt1, groups0, res_scale, sol_scale, blk);
  else
    colour_pass_lines<D, K, T, MODE, PPW>(smem, b, x, n1d, p0, p1, p2, cnt0, cnt1, groups0, res_scale, sol_scale,
                                          blk);
}

template <int D, int K, typename T, int MODE, int PPW>
__global__ __launch_bounds__((ColourNT<D, K, T, MODE, PPW>::value)) void colour_pass_kernel(
    const T* __restrict__ b, T* __restrict__ x, long long n1d, int p0, int p1, int p2, int cnt0, int cnt1,
    int groups0, T res_scale, T sol_scale) {
  __shared__ __align__(16) T smem[ColourLds<D, K, T, MODE, PPW>::value];
  colour_pass_block<D, K, T, MODE, PPW>(smem, b, x, n1d, p0, p1, p2, cnt0, cnt1, groups0, res_scale, sol_scale,
                                  xcd_remap(blockIdx.x, gridDim.x));
}

// Several colour passes of the same (dim, degree, precision, colour) on different vectors and
// levels in one launch: entry e owns blocks [begin[e], begin[e+1]).
template <int D, int K, typename T, int MODE, int PPW>
__global__ __launch_bounds__((ColourNT<D, K, T, MODE, PPW>::value)) void colour_pass_group_kernel(ColourPassGroup grp) {
  __shared__ __align__(16) T smem[ColourLds<D, K, T, MODE, PPW>::value];
  const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
  int e = 0;
  while (e + 1 < grp.n && (unsigned)grp.e[e + 1].block_begin <= g) ++e;
  const ColourPassDesc& d = grp.e[e];
  colour_pass_block<D, K, T, MODE, PPW>(smem, (const T*)d.b, (T*)d.x, d.n1d, d.p[0], d.p[1], d.p[2], d.cnt0, d.cnt1,
                                  d.groups0, (T)d.res_scale, (T)d.sol_scale, g - (unsigned)d.block_begin);
}

// ------------------------------------------------------------------ host side

// Patch grid of one colour on one level: parities, counts per axis, workgroups along x0.
template <int D, int K>
struct ColourGrid {
  int p[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  int groups0 = 0;
  long long blocks = 0;
  bool ok = true;  // the 32-bit block (byte) offsets of the kernel are valid
  ColourGrid(const LevelGeom& g, int colour, int PPW = SmootherShape<D, K>::PPW) {
    const int half = (int)(g.ncells / 2);
    for (int a = 0; a < D; ++a) {
      p[a] = (colour >> a) & 1;
      cnt[a] = half - p[a];
    }
    for (int a = 0; a < D; ++a)
      if (cnt[a] <= 0) return;  // empty colour (coarsest level)
    groups0 = (cnt[0] + PPW - 1) / PPW;
    blocks = (long long)groups0 * cnt[1] * (D == 3 ? cnt[2] : 1);
    constexpr long long n = 2 * K + 1;
    const long long span = (D == 3 ? (n - 1) * g.n1d * g.n1d : 0) + (n - 1) * g.n1d + 2 * K * PPW + 1;
    ok = blocks <= 0x7fffffffLL && span < (1LL << 29);  // byte offsets of 8-byte words fit in 32 bits
  }
};

template <int D, int K, typename T, int MODE, int PPW>
static hipError_t launch_shape(const LevelGeom& g, const ColourGrid<D, K>& cg, const void* b, void* x,
                               hipStream_t st) {
  constexpr int NT = ColourNT<D, K, T, MODE, PPW>::value;
  // Abar_h = h^(d-2) Abar_1 ; A_j,h^{-1} = h^(2-d) A_j,1^{-1}
  const T res_scale = (T)(D == 3 ? g.h : 1.0);
  const T sol_scale = (T)(D == 3 ? 1.0 / g.h : 1.0);
  hipLaunchKernelGGL((colour_pass_kernel<D, K, T, MODE, PPW>), dim3((unsigned)cg.blocks), dim3(NT), 0, st,
                     (const T*)b, (T*)x, g.n1d, cg.p[0], cg.p[1], cg.p[2], cg.cnt[0], cg.cnt[1], cg.groups0,
                     res_scale, sol_scale);
  return hipGetLastError();
}

// The wide shape's launch: enough workgroups to leave the small-launch regime and few idle patch
// slots at row ends.
template <int D, int K>
static bool wide_fits(const ColourGrid<D, K>& cw) {
  return cw.ok && cw.blocks >= kLatencyBlocks &&
         (double)(cw.groups0 * kWidePPW - cw.cnt[0]) <= kWideIdle * (double)cw.cnt[0];
}

template <int D, int K, typename T, int MODE>
static hipError_t launch_one(const LevelGeom& g, int colour, const void* b, void* x, hipStream_t st) {
  constexpr int PPW = ColourShape<D, K, T, MODE>::PPW, LPPW = LatencyPPW<D, K>::value;
  if constexpr (HasWideForm<D, K, T, MODE>::value) {
    const ColourGrid<D, K> cw(g, colour, kWidePPW);
    if (wide_fits(cw)) return launch_shape<D, K, T, MODE, kWidePPW>(g, cw, b, x, st);
  }
  const ColourGrid<D, K> cg(g, colour, PPW);
  if (!cg.ok) return hipErrorInvalidConfiguration;
  if (cg.blocks == 0) return hipSuccess;
  if constexpr (LPPW < PPW) {
    if (cg.blocks < kLatencyBlocks) {
      const ColourGrid<D, K> cl(g, colour, LPPW);
      if (!cl.ok) return hipErrorInvalidConfiguration;
      return launch_shape<D, K, T, MODE, LPPW>(g, cl, b, x, st);
    }
  }
  return launch_shape<D, K, T, MODE, PPW>(g, cg, b, x, st);
}

// True when a stand-alone pass of this colour and level runs the matrix-core form (launch_one: the
// default shape, not the small-launch one).  A packed launch must give each member the arithmetic of
// its stand-alone pass, so that a result does not depend on the requests it is served with.
template <int D, int K, typename T, int MODE>
static bool member_uses_mfma(const LevelGeom& g, int colour) {
  if constexpr (!UsesMfma<D, K, T, MODE>::value) {
    return false;
  } else {
    const ColourGrid<D, K> cg(g, colour, kMfmaPPW);
    return cg.blocks >= kLatencyBlocks;
  }
}

// The members with mfma == member_uses_mfma, in launches of PPW patches per workgroup.
template <int D, int K, typename T, int MODE, int PPW>
static hipError_t launch_group_form(int colour, const ColourPassMember* mem, int nm, bool mfma, hipStream_t st) {
  constexpr int NT = ColourNT<D, K, T, MODE, PPW>::value;
  ColourPassGroup grp;
  grp.n = 0;
  long long total = 0;
  auto flush = [&]() -> hipError_t {
    if (grp.n == 0) return hipSuccess;
    hipLaunchKernelGGL((colour_pass_group_kernel<D, K, T, MODE, PPW>), dim3((unsigned)total), dim3(NT), 0, st, grp);
    grp.n = 0;
    total = 0;
    return hipGetLastError();
  };
  for (int i = 0; i < nm; ++i) {
    if (member_uses_mfma<D, K, T, MODE>(mem[i].g, colour) != mfma) continue;
    const ColourGrid<D, K> cg(mem[i].g, colour, PPW);
    if (!cg.ok) return hipErrorInvalidConfiguration;
    if (cg.blocks == 0) continue;
    if (grp.n == kMaxGroup || total + cg.blocks > 0x7fffffffLL) {
      hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
    ColourPassDesc& d = grp.e[grp.n++];
    d.b = mem[i].b;
    d.x = mem[i].x;
    d.n1d = mem[i].g.n1d;
    d.p[0] = cg.p[0];
    d.p[1] = cg.p[1];
    d.p[2] = cg.p[2];
    d.cnt0 = cg.cnt[0];
    d.cnt1 = cg.cnt[1];
    d.groups0 = cg.groups0;
    d.block_begin = (int)total;
    d.res_scale = D == 3 ? mem[i].g.h : 1.0;
    d.sol_scale = D == 3 ? 1.0 / mem[i].g.h : 1.0;
    total += cg.blocks;
  }
  return flush();
}

template <int D, int K, typename T, int MODE>
static hipError_t launch_group(int colour, const ColourPassMember* mem, int nm, hipStream_t st) {
  constexpr int PPW = SmootherShape<D, K>::PPW;
  if constexpr (UsesMfma<D, K, T, MODE>::value) {
    hipError_t e = launch_group_form<D, K, T, MODE, kMfmaPPW>(colour, mem, nm, true, st);
    if (e != hipSuccess) return e;
  }
  return launch_group_form<D, K, T, MODE, PPW>(colour, mem, nm, false, st);
}

template <int D, int K, typename T>
static hipError_t dispatch_mode(const LevelGeom& g, int mode, int colour, const void* b, void* x, hipStream_t st) {
  switch (mode) {
    case kModeMultiplicative: return launch_one<D, K, T, kModeMultiplicative>(g, colour, b, x, st);
    case kModeAdditive: return launch_one<D, K, T, kModeAdditive>(g, colour, b, x, st);
    case kModeBoundary: return launch_one<D, K, T, kModeBoundary>(g, colour, b, x, st);
    case kModeMfma:
      if constexpr (HasMfmaForm<D, K, T>::value) return launch_one<D, K, T, kModeMfma>(g, colour, b, x, st);
      return launch_one<D, K, T, kModeMultiplicative>(g, colour, b, x, st);
    case kModeZero:
      if (colour != 0) return hipErrorInvalidValue;  // only colour 0's closures tile the grid
      return launch_one<D, K, T, kModeZero>(g, colour, b, x, st);
  }
  return hipErrorInvalidValue;
}

template <int D, int K>
static hipError_t dispatch_prec(const LevelGeom& g, int prec, int mode, int colour, const void* b, void* x,
                                hipStream_t st) {
  return prec == 0 ? dispatch_mode<D, K, double>(g, mode, colour, b, x, st)
                   : dispatch_mode<D, K, float>(g, mode, colour, b, x, st);
}

template <int D>
static hipError_t dispatch_k(const LevelGeom& g, int prec, int mode, int colour, const void* b, void* x,
                             hipStream_t st) {
  switch (g.k) {
    case 1: return dispatch_prec<D, 1>(g, prec, mode, colour, b, x, st);
    case 2: return dispatch_prec<D, 2>(g, prec, mode, colour, b, x, st);
    case 3: return dispatch_prec<D, 3>(g, prec, mode, colour, b, x, st);
    case 4: return dispatch_prec<D, 4>(g, prec, mode, colour, b, x, st);
    case 5: return dispatch_prec<D, 5>(g, prec, mode, colour, b, x, st);
    case 6: return dispatch_prec<D, 6>(g, prec, mode, colour, b, x, st);
    case 7: return dispatch_prec<D, 7>(g, prec, mode, colour, b, x, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_colour_pass(const LevelGeom& g, int prec, int mode, int colour, const void* b, void* x,
                              hipStream_t st) {
  return g.dim == 2 ? dispatch_k<2>(g, prec, mode, colour, b, x, st) : dispatch_k<3>(g, prec, mode, colour, b, x, st);
}

template <int D, int K>
static hipError_t group_prec(int prec, int mode, int colour, const ColourPassMember* m, int nm, hipStream_t st) {
  if (mode == kModeAdditive)
    return prec == 0 ? launch_group<D, K, double, kModeAdditive>(colour, m, nm, st)
                     : launch_group<D, K, float, kModeAdditive>(colour, m, nm, st);
  if (mode == kModeMultiplicative)
    return prec == 0 ? launch_group<D, K, double, kModeMultiplicative>(colour, m, nm, st)
                     : launch_group<D, K, float, kModeMultiplicative>(colour, m, nm, st);
  if (mode == kModeBoundary)
    return prec == 0 ? launch_group<D, K, double, kModeBoundary>(colour, m, nm, st)
                     : launch_group<D, K, float, kModeBoundary>(colour, m, nm, st);
  if (mode == kModeZero) {
    if (colour != 0) return hipErrorInvalidValue;
    return prec == 0 ? launch_group<D, K, double, kModeZero>(colour, m, nm, st)
                     : launch_group<D, K, float, kModeZero>(colour, m, nm, st);
  }
  if (mode == kModeMfma) {
    if constexpr (HasMfmaForm<D, K, float>::value)
      if (prec == 1) return launch_group<D, K, float, kModeMfma>(colour, m, nm, st);
    return prec == 0 ? launch_group<D, K, double, kModeMultiplicative>(colour, m, nm, st)
                     : launch_group<D, K, float, kModeMultiplicative>(colour, m, nm, st);
  }
  return hipErrorInvalidValue;
}

template <int D>
static hipError_t group_k(int k, int prec, int mode, int colour, const ColourPassMember* m, int nm, hipStream_t st) {
  switch (k) {
    case 1: return group_prec<D, 1>(prec, mode, colour, m, nm, st);
    case 2: return group_prec<D, 2>(prec, mode, colour, m, nm, st);
    case 3: return group_prec<D, 3>(prec, mode, colour, m, nm, st);
    case 4: return group_prec<D, 4>(prec, mode, colour, m, nm, st);
    case 5: return group_prec<D, 5>(prec, mode, colour, m, nm, st);
    case 6: return group_prec<D, 6>(prec, mode, colour, m, nm, st);
    case 7: return group_prec<D, 7>(prec, mode, colour, m, nm, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_colour_pass_group(int dim, int k, int prec, int mode, int colour, const ColourPassMember* members,
                                    int n_members, hipStream_t st) {
  return dim == 2 ? group_k<2>(k, prec, mode, colour, members, n_members, st)
                  : group_k<3>(k, prec, mode, colour, members, n_members, st);
}

// ------------------------------------------------------------ host-side launch geometry

namespace {

// Every workgroup of one colour's launch with PPW patches per workgroup: its patches lie in the
// colour and inside the grid, the workgroups cover the colour's patches once, and the farthest
// closure node of a workgroup is within the kernels' 32-bit byte offsets (8-byte words).
template <int D, int K, int PPW>
bool colour_shape_ok(const LevelGeom& g, int colour, long long* nblk, std::string* why) {
  const ColourGrid<D, K> cg(g, colour, PPW);
  if (cg.blocks == 0) return true;
  const std::string tag = "colour " + std::to_string(colour) + ", " + std::to_string(PPW) + " patches per workgroup: ";
  if (!cg.ok) return *why = tag + "launch refused (offsets or grid beyond 32 bits)", false;
  const long long n1d = g.n1d, nc = g.ncells, span = 2LL * K;
  long long patches = 0;
  for (long long b = 0; b < cg.blocks; ++b) {
    const ColourBlock cb = colour_block<D, K, PPW>((unsigned)b, cg.p[0], cg.p[1], cg.p[2], cg.cnt[0], cg.cnt[1],
                                                   cg.groups0);
    if (cb.count < 1 || cb.count > PPW) return *why = tag + "workgroup without patches", false;
    const long long s[3] = {cb.s0, cb.s1, cb.s2};
    for (int a = 0; a < D; ++a) {
      const long long v = s[a] / K + 1;  // vertex of the workgroup's first patch
      if (s[a] % K != 0 || v < 1 || v > nc - 1 || ((v - 1) & 1) != cg.p[a])
        return *why = tag + "patch outside the colour", false;
    }
    if (s[0] / K + 1 + 2LL * (cb.count - 1) > nc - 1) return *why = tag + "patch past the last vertex", false;
    if (cb.s0 + span * cb.count > n1d - 1 || cb.s1 + span > n1d - 1 || (D == 3 && cb.s2 + span > n1d - 1))
      return *why = tag + "closure outside the grid", false;
    const long long far = (D == 3 ? span * n1d * n1d : 0) + span * n1d + span * cb.count;
    if (far * 8 >= (1LL << 32)) return *why = tag + "closure offsets beyond 32 bits", false;
    patches += cb.count;
  }
  const long long want = (long long)cg.cnt[0] * cg.cnt[1] * (D == 3 ? cg.cnt[2] : 1);
  if (patches != want) return *why = tag + "workgroups do not cover the colour once", false;
  *nblk += cg.blocks;
  return true;
}

template <int D, int K>
bool colour_launches_ok(const LevelGeom& g, long long* nblk, std::string* why) {
  for (int c = 0; c < (1 << D); ++c) {
    if (!colour_shape_ok<D, K, SmootherShape<D, K>::PPW>(g, c, nblk, why)) return false;
    if (!colour_shape_ok<D, K, LatencyPPW<D, K>::value>(g, c, nblk, why)) return false;
    if constexpr (HasMfmaForm<D, K, float>::value)
      if (!colour_shape_ok<D, K, kMfmaPPW>(g, c, nblk, why)) return false;
    if constexpr (HasWideForm<D, K, float, kModeMultiplicative>::value)
      if (!colour_shape_ok<D, K, kWidePPW>(g, c, nblk, why)) return false;
  }
  return true;
}

}  // namespace

bool check_colour_launches(const LevelGeom& g, long long* blocks, std::string* why) {
  switch (g.dim * 10 + g.k) {
    case 21: return colour_launches_ok<2, 1>(g, blocks, why);
    case 22: return colour_launches_ok<2, 2>(g, blocks, why);
    case 23: return colour_launches_ok<2, 3>(g, blocks, why);
    case 24: return colour_launches_ok<2, 4>(g, blocks, why);
    case 25: return colour_launches_ok<2, 5>(g, blocks, why);
    case 26: return colour_launches_ok<2, 6>(g, blocks, why);
    case 27: return colour_launches_ok<2, 7>(g, blocks, why);
    case 31: return colour_launches_ok<3, 1>(g, blocks, why);
    case 32: return colour_launches_ok<3, 2>(g, blocks, why);
    case 33: return colour_launches_ok<3, 3>(g, blocks, why);
    case 34: return colour_launches_ok<3, 4>(g, blocks, why);
    case 35: return colour_launches_ok<3, 5>(g, blocks, why);
    case 36: return colour_launches_ok<3, 6>(g, blocks, why);
    case 37: return colour_launches_ok<3, 7>(g, blocks, why);
  }
  *why = "unsupported (dim, degree)";
  return false;
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
