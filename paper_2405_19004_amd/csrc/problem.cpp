// Level hierarchy, V-cycle (Alg. 1) and preconditioned CG drivers.  The host
// only sequences launches (Sec. 3: building blocks launched one after the
// other); all vectors stay resident on the device during a solve (Sec. 3.1).
#include "problem.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.hpp"

#define VPS_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return Status{-3, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define VPS_TRY(expr)                 \
  do {                                \
    Status s_ = (expr);               \
    if (s_.code != 0) return s_;      \
  } while (0)

namespace vps {

// Kernel mode of the V-cycle smoothing steps.
// Smoother mode of the Separate form (not a kernel mode): per colour, the global residual by the
// operator kernel, then the local solves of the additive kernel on that residual.
constexpr int kSmoothSeparate = 3;
inline int vcycle_mode(const Problem* p) {
  return p->separate_smoother   ? kSmoothSeparate
         : p->boundary_smoother ? kModeBoundary
         : p->mfma_smoother     ? kModeMfma
                                : kModeMultiplicative;
}

long long level_nodes(int dim, int k, int level) {
  long long n = (long long)k * (1LL << level) + 1;
  return dim == 2 ? n * n : n * n * n;
}

LevelGeom make_geom(int dim, int k, int level) {
  LevelGeom g;
  g.dim = dim;
  g.k = k;
  g.level = level;
  g.ncells = 1LL << level;
  g.n1d = (long long)k * g.ncells + 1;
  g.h = 1.0 / (double)g.ncells;
  return g;
}

namespace {

struct Plan {
  // byte sizes of every allocation in creation order
  std::vector<size_t> sizes;
};

// Partial sums of the reductions: the vector reductions' pairs, and on the finest level one per
// workgroup of the fused operator forms.
long long partial_count(int dim, int k, int L) {
  return std::max<long long>(2LL * reduction_parts(), fused_reduction_parts(make_geom(dim, k, L)));
}

// The allocation plan is the single source of the footprint and of create_problem.
Plan plan(int dim, int k, int L, unsigned flags) {
  Plan pl;
  const bool h64 = flags & 0x1u, h32 = flags & 0x2u, solver = !(flags & 0x4u);
  for (int lvl = 1; lvl <= L; ++lvl) {
    const size_t N = (size_t)level_nodes(dim, k, lvl);
    for (int prec = 0; prec < 2; ++prec) {
      const bool want = prec == 0 ? h64 : h32;
      if (!want) continue;
      const size_t es = prec == 0 ? 8 : 4;
      const bool bx = lvl < L || prec == 1;
      if (bx) {
        pl.sizes.push_back(N * es);  // b
        pl.sizes.push_back(N * es);  // x
      }
      pl.sizes.push_back(N * es);  // r (V-cycle residual; the Separate smoother's residual on every level)
      if (lvl >= 2 && dim == 3) pl.sizes.push_back((size_t)restrict_scratch_elems(dim, k, lvl) * es);  // restriction scratch
    }
  }
  if (h32) {
    const size_t N1 = (size_t)level_nodes(dim, k, 1);
    pl.sizes.push_back(N1 * 8);
    pl.sizes.push_back(N1 * 8);
  }
  if (solver) {
    // r, z, p, q; z only with the FP64 hierarchy: a mixed solve reads the FP32 V-cycle output
    const size_t N = (size_t)level_nodes(dim, k, L);
    for (int i = 0; i < (h64 ? 4 : 3); ++i) pl.sizes.push_back(N * 8);
  }
  pl.sizes.push_back(kScCount * 8);
  pl.sizes.push_back((size_t)partial_count(dim, k, L) * 8);
  pl.sizes.push_back(256);  // flag
  return pl;
}

size_t round_up(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t footprint_bytes(int dim, int degree, int L, unsigned flags) {
  Plan pl = plan(dim, degree, L, flags);
  size_t t = 0;
  for (size_t s : pl.sizes) t += round_up(s);
  return t;
}

Problem::~Problem() {
  if (stream) hipStreamSynchronize(stream);
  if (graph_stream) (void)hipStreamSynchronize(graph_stream);
  for (hipGraphExec_t g : precond_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (graph_in) (void)hipEventDestroy(graph_in);
  if (graph_out) (void)hipEventDestroy(graph_out);
  if (graph_stream) (void)hipStreamDestroy(graph_stream);
  for (void* a : allocs) hipFree(a);
  if (host_sc) hipHostFree(host_sc);
  if (host_bad) hipHostFree(host_bad);
}

bool Problem::has(int prec) const { return prec == 0 ? (flags & 0x1u) : (flags & 0x2u); }

Status create_problem(int dim, int k, int L, unsigned flags, hipStream_t st, Problem** out) {
  static bool tables_ready = false;
  if (!tables_ready) {
    VPS_HIP(init_smoother_tables());
    tables_ready = true;
  }
  Problem* p = new Problem();
  p->dim = dim;
  p->k = k;
  p->L = L;
  p->flags = flags;
  p->stream = st;
  p->post_same_order = flags & 0x8u;
  p->boundary_smoother = flags & 0x10u;
  p->separate_smoother = flags & 0x40u;
  p->mfma_smoother = flags & 0x80u;
  p->use_graphs = flags & 0x20u;
  p->lv.resize(L + 1);
  Plan pl = plan(dim, k, L, flags);
  std::vector<void*> ptrs;
  for (size_t s : pl.sizes) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, round_up(s));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete p;
      return Status{-2, "hipMalloc of " + std::to_string(round_up(s)) + " bytes failed"};
    }
    p->allocs.push_back(d);
    p->bytes += round_up(s);
    e = hipMemsetAsync(d, 0, round_up(s), st);
    if (e != hipSuccess) {
      delete p;
      return Status{-3, std::string("hipMemsetAsync: ") + hipGetErrorString(e)};
    }
  }
  // hand out in plan order
  size_t idx = 0;
  const bool h64 = flags & 0x1u, h32 = flags & 0x2u, solver = !(flags & 0x4u);
  for (int lvl = 1; lvl <= L; ++lvl) {
    LevelBuffers& B = p->lv[lvl];
    B.g = make_geom(dim, k, lvl);
    B.N = level_nodes(dim, k, lvl);
    for (int prec = 0; prec < 2; ++prec) {
      const bool want = prec == 0 ? h64 : h32;
      if (!want) continue;
      const bool bx = lvl < L || prec == 1;
      if (bx) {
        B.b[prec] = p->allocs[idx++];
        B.x[prec] = p->allocs[idx++];
      }
      B.r[prec] = p->allocs[idx++];
      if (lvl >= 2 && dim == 3) B.t[prec] = p->allocs[idx++];
    }
  }
  if (h32) {
    p->c64_b = (double*)p->allocs[idx++];
    p->c64_x = (double*)p->allocs[idx++];
  }
  if (solver) {
    p->r = (double*)p->allocs[idx++];
    if (h64) p->z = (double*)p->allocs[idx++];
    p->p = (double*)p->allocs[idx++];
    p->q = (double*)p->allocs[idx++];
  }
  p->sc = (double*)p->allocs[idx++];
  p->partial = (double*)p->allocs[idx++];
  p->n_partial = partial_count(dim, k, L);
  p->bad = (int*)p->allocs[idx++];
  if (hipHostMalloc((void**)&p->host_sc, kScCount * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->host_bad, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return Status{-2, "hipHostMalloc failed"};
  }
  VPS_HIP(hipStreamSynchronize(st));
  *out = p;
  return Status::ok();
}

// ------------------------------------------------------------------ smoothing

Status colour_pass(Problem* p, int level, int prec, int mode, int colour, const void* b, void* x) {
  if (mode == kSmoothSeparate) {
    // same-colour patches are disjoint, so one residual r = b - A x (before the colour) serves them
    // all and x^I += A_j^{-1} r^I is the multiplicative update
    void* r = p->lv[level].r[prec];
    if (!r) return Status{-1, "the Separate smoother needs the matching hierarchy flag"};
    VPS_HIP(launch_operator(p->geom(level), prec, x, b, r, p->stream));
    VPS_HIP(launch_colour_pass(p->geom(level), prec, kModeAdditive, colour, r, x, p->stream));
    return Status::ok();
  }
  VPS_HIP(launch_colour_pass(p->geom(level), prec, mode, colour, b, x, p->stream));
  return Status::ok();
}

Status smoother(Problem* p, int level, int prec, int mode, bool reverse, const void* b, void* x, bool x_zero) {
  const int nc = 1 << p->dim;
  for (int i = 0; i < nc; ++i) {
    const int c = reverse ? nc - 1 - i : i;
    // on x = 0 the first multiplicative colour reduces to x^I = A_j^{-1} b^I (residual = b,
    // x^B = 0): the additive kernel gives the same values without forming the residual; for colour
    // 0 the from-zero kernel also writes the zeros of the rest of the grid, so x may hold anything
    const int m = (i == 0 && x_zero && mode != kModeAdditive) ? (c == 0 ? kModeZero : kModeAdditive) : mode;
    VPS_TRY(colour_pass(p, level, prec, m, c, b, x));
  }
  return Status::ok();
}

Status coarse_solve(Problem* p, int prec, const void* b, void* x) {
  const LevelGeom& g = p->geom(1);
  const long long N = p->lv[1].N;
  if (prec == 0) {
    VPS_HIP(launch_fill(0, x, N, 0.0, p->stream));
    VPS_HIP(launch_colour_pass(g, 0, kModeMultiplicative, 0, b, x, p->stream));
    return Status::ok();
  }
  if (!p->c64_b) return Status{-1, "FP32 coarse solve needs the FP32 hierarchy"};
  VPS_HIP(launch_widen_zero(static_cast<const float*>(b), p->c64_b, p->c64_x, N, p->stream));
  VPS_HIP(launch_colour_pass(g, 0, kModeMultiplicative, 0, p->c64_b, p->c64_x, p->stream));
  VPS_HIP(launch_cast(0, p->c64_x, x, N, p->stream));
  return Status::ok();
}

Status vcycle_top(Problem* p, int prec, int top, const void* bT, void* xT, bool top_zero) {
  if (!p->has(prec)) return Status{-1, "V-cycle precision was not requested at creation"};
  if (top == 1) return coarse_solve(p, prec, bT, xT);
  const bool post_rev = !p->post_same_order;
  // descend
  for (int lvl = top; lvl >= 2; --lvl) {
    const void* b = lvl == top ? bT : p->lv[lvl].b[prec];
    void* x = lvl == top ? xT : p->lv[lvl].x[prec];
    // below the top, x starts from 0: the restriction into this level zeroed it
    VPS_TRY(smoother(p, lvl, prec, vcycle_mode(p), false, b, x, lvl < top || top_zero));
    VPS_HIP(launch_operator(p->geom(lvl), prec, x, b, p->lv[lvl].r[prec], p->stream));
    VPS_HIP(launch_restrict(p->geom(lvl), prec, p->lv[lvl].r[prec], p->lv[lvl - 1].b[prec], p->lv[lvl].t[prec],
                            p->stream, lvl - 1 >= 2 ? p->lv[lvl - 1].x[prec] : nullptr));
  }
  VPS_TRY(coarse_solve(p, prec, p->lv[1].b[prec], p->lv[1].x[prec]));
  // ascend
  for (int lvl = 2; lvl <= top; ++lvl) {
    const void* b = lvl == top ? bT : p->lv[lvl].b[prec];
    void* x = lvl == top ? xT : p->lv[lvl].x[prec];
    VPS_HIP(launch_prolongate_add(p->geom(lvl), prec, p->lv[lvl - 1].x[prec], x, p->stream));
    VPS_TRY(smoother(p, lvl, prec, vcycle_mode(p), post_rev, b, x));
  }
  return Status::ok();
}

Status vcycle(Problem* p, int prec, const void* bL, void* xL) { return vcycle_top(p, prec, p->L, bL, xL, false); }

// ------------------------------------------------------------------------ FMG

namespace {

// *out_slot <- ||v||^2 over the interior nodes of the finest level (v in `prec`); the FP64 copy
// goes to p->q (p->p is scratch: FMG does not run CG).  Sets p->bad on a non-finite entry.
Status interior_norm2(Problem* p, int prec, const void* v, double* out_slot) {
  const LevelGeom& g = p->geom(p->L);
  const double* src = static_cast<const double*>(v);
  if (prec == 1) {
    VPS_HIP(launch_cast(1, v, p->p, p->lv[p->L].N, p->stream));
    src = p->p;
  }
  VPS_HIP(launch_copy_interior_norm(p->dim, g.n1d, src, p->q, p->partial, out_slot, p->bad, p->stream));
  return Status::ok();
}

// *out_slot <- ||b - A x||^2 on the finest level (residual formed in `prec`).  The residual
// buffers keep zero boundary entries: the operator kernel writes interior nodes only.
Status residual_norm2(Problem* p, int prec, const void* b, const void* x, double* out_slot) {
  const LevelGeom& g = p->geom(p->L);
  const long long N = p->lv[p->L].N;
  if (prec == 0) {
    VPS_HIP(launch_operator(g, 0, x, b, p->q, p->stream));
  } else {
    void* r32 = p->lv[p->L].r[1];
    if (!r32) {  // single-level hierarchy: FP32 residual in the front half of p (scratch here)
      r32 = p->p;
      VPS_HIP(launch_fill(1, r32, N, 0.0, p->stream));
    }
    VPS_HIP(launch_operator(g, 1, x, b, r32, p->stream));
    VPS_HIP(launch_cast(1, r32, p->q, N, p->stream));
  }
  VPS_HIP(launch_dot2(p->q, p->q, nullptr, nullptr, N, p->partial, out_slot, p->stream));
  return Status::ok();
}

Status fetch_scalars(Problem* p) {
  VPS_HIP(hipMemcpyAsync(p->host_sc, p->sc, kScCount * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  VPS_HIP(hipMemcpyAsync(p->host_bad, p->bad, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  VPS_HIP(hipStreamSynchronize(p->stream));
  return Status::ok();
}

}  // namespace

Status fmg(Problem* p, int prec, const void* const* b_levels, void* x, double eps, int maxit, SolveStats* out) {
  if (!p->r) return Status{-1, "FMG needs the solver vectors (problem created without them)"};
  if (!p->has(prec)) return Status{-1, "FMG precision was not requested at creation"};
  const int L = p->L;
  SolveStats st;
  VPS_HIP(hipMemsetAsync(p->bad, 0, sizeof(int), p->stream));
  VPS_TRY(interior_norm2(p, prec, b_levels[L - 1], p->sc + kScBB));
  // nested iteration: exact solve on level 1, then one V-cycle per level from the prolongated
  // coarser solution
  auto level_x = [&](int lvl) -> void* { return lvl == L ? x : p->lv[lvl].x[prec]; };
  VPS_TRY(coarse_solve(p, prec, b_levels[0], level_x(1)));
  for (int lvl = 2; lvl <= L; ++lvl) {
    VPS_HIP(launch_fill(prec, level_x(lvl), p->lv[lvl].N, 0.0, p->stream));
    VPS_HIP(launch_prolongate_add(p->geom(lvl), prec, level_x(lvl - 1), level_x(lvl), p->stream));
    VPS_TRY(vcycle_top(p, prec, lvl, b_levels[lvl - 1], level_x(lvl), false));
  }
  VPS_TRY(residual_norm2(p, prec, b_levels[L - 1], x, p->sc + kScTrue));
  VPS_TRY(fetch_scalars(p));
  const double d0 = std::sqrt(p->host_sc[kScBB]);
  if (*p->host_bad || !std::isfinite(d0)) {
    st.status = -6;
    if (out) *out = st;
    return Status::ok();
  }
  double delta = std::sqrt(p->host_sc[kScTrue]);
  // further V-cycles on the finest level until the residual has dropped by eps
  while (std::isfinite(delta) && delta > eps * d0 && st.iterations < maxit) {
    VPS_TRY(vcycle_top(p, prec, L, b_levels[L - 1], x, false));
    VPS_TRY(residual_norm2(p, prec, b_levels[L - 1], x, p->sc + kScTrue));
    VPS_TRY(fetch_scalars(p));
    delta = std::sqrt(p->host_sc[kScTrue]);
    st.iterations += 1;
  }
  st.rel_residual = st.true_rel_residual = d0 > 0.0 ? delta / d0 : delta;
  st.status = !std::isfinite(delta) ? -6 : delta > eps * d0 ? -4 : 0;
  if (out) *out = st;
  return Status::ok();
}

Status vcycle_group(Problem* const* ps, int n, int prec, const void* const* bL, void* const* xL, bool top_zero) {
  if (n <= 0) return Status::ok();
  int Lmax = 0;
  for (int i = 0; i < n; ++i) {
    if (!ps[i]->has(prec)) return Status{-1, "V-cycle precision was not requested at creation"};
    if (ps[i]->dim != ps[0]->dim || ps[i]->k != ps[0]->k || ps[i]->stream != ps[0]->stream ||
        ps[i]->post_same_order != ps[0]->post_same_order || vcycle_mode(ps[i]) != vcycle_mode(ps[0]))
      return Status{-1, "grouped V-cycle needs one dim, degree, stream, colour order and smoother kernel"};
    Lmax = ps[i]->L > Lmax ? ps[i]->L : Lmax;
  }
  const int dim = ps[0]->dim, k = ps[0]->k, nc = 1 << dim;
  const bool post_rev = !ps[0]->post_same_order;
  hipStream_t st = ps[0]->stream;
  auto level_b = [&](int i, int lvl) -> const void* { return lvl == ps[i]->L ? bL[i] : ps[i]->lv[lvl].b[prec]; };
  auto level_x = [&](int i, int lvl) -> void* { return lvl == ps[i]->L ? xL[i] : ps[i]->lv[lvl].x[prec]; };
  std::vector<ColourPassMember> mem, sep;
  // x_zero: every member's x is 0 on entry (the first colour then needs no residual, as in smoother())
  auto smooth = [&](int lvl, bool reverse, bool x_zero) -> Status {
    mem.clear();
    for (int i = 0; i < n; ++i)
      if (ps[i]->L >= lvl) mem.push_back({ps[i]->geom(lvl), level_b(i, lvl), level_x(i, lvl)});
    for (int j = 0; j < nc; ++j) {
      const int c = reverse ? nc - 1 - j : j;
      int mode = (j == 0 && x_zero) ? (c == 0 ? kModeZero : kModeAdditive) : vcycle_mode(ps[0]);
      if (mode == kSmoothSeparate) {
        // residual of every member, then the packed local solves on it
        sep.assign(mem.begin(), mem.end());
        int m = 0;
        for (int i = 0; i < n; ++i) {
          if (ps[i]->L < lvl) continue;
          VPS_HIP(launch_operator(ps[i]->geom(lvl), prec, level_x(i, lvl), level_b(i, lvl), ps[i]->lv[lvl].r[prec], st));
          sep[m++].b = ps[i]->lv[lvl].r[prec];
        }
        VPS_HIP(launch_colour_pass_group(dim, k, prec, kModeAdditive, c, sep.data(), (int)sep.size(), st));
        continue;
      }
      VPS_HIP(launch_colour_pass_group(dim, k, prec, mode, c, mem.data(), (int)mem.size(), st));
    }
    return Status::ok();
  };
  for (int lvl = Lmax; lvl >= 2; --lvl) {
    // levels below a member's top start from 0 (the restriction into them zeroed x)
    VPS_TRY(smooth(lvl, false, top_zero));
    for (int i = 0; i < n; ++i) {
      if (ps[i]->L < lvl) continue;
      Problem* p = ps[i];
      VPS_HIP(launch_operator(p->geom(lvl), prec, level_x(i, lvl), level_b(i, lvl), p->lv[lvl].r[prec], st));
      VPS_HIP(launch_restrict(p->geom(lvl), prec, p->lv[lvl].r[prec], p->lv[lvl - 1].b[prec], p->lv[lvl].t[prec], st,
                              lvl - 1 >= 2 ? p->lv[lvl - 1].x[prec] : nullptr));
    }
  }
  for (int i = 0; i < n; ++i) VPS_TRY(coarse_solve(ps[i], prec, level_b(i, 1), level_x(i, 1)));
  for (int lvl = 2; lvl <= Lmax; ++lvl) {
    for (int i = 0; i < n; ++i)
      if (ps[i]->L >= lvl)
        VPS_HIP(launch_prolongate_add(ps[i]->geom(lvl), prec, ps[i]->lv[lvl - 1].x[prec], level_x(i, lvl), st));
    VPS_TRY(smooth(lvl, post_rev, false));
  }
  return Status::ok();
}

// ------------------------------------------------------------------------ CG

namespace {

// The preconditioned residual of a mixed solve: the FP32 V-cycle's result on the finest level (it
// stays there until the next preconditioner application); null in FP64 mode, where z is p->z.
const float* cg_z32(const Problem* p, int mode) {
  return mode == 1 ? static_cast<const float*>(p->lv[p->L].x[1]) : nullptr;
}

// z = M r with the problem's CG vectors, and sc[RZNew] = r.z.  Mixed mode: the FP32 copy of r
// must already be in the level-L FP32 rhs (cg_update or pcg_begin writes it), and z stays the FP32
// result in the level-L FP32 iterate (cg_z32): its consumers widen it exactly as they read it.
Status precondition_launch(Problem* p, int mode) {
  const long long N = p->lv[p->L].N;
  // z = V(r) from z = 0: the V-cycle's first pass (colour 0 from zero, or the coarse solve on a
  // one-level hierarchy) writes every node of z, so z is not cleared first
  if (mode == 0) {
    VPS_TRY(vcycle_top(p, 0, p->L, p->r, p->z, true));
    VPS_HIP(launch_dot2(p->r, p->z, nullptr, nullptr, N, p->partial, p->sc + kScRZNew, p->stream));
    return Status::ok();
  }
  LevelBuffers& B = p->lv[p->L];
  VPS_TRY(vcycle_top(p, 1, p->L, B.b[1], B.x[1], true));
  VPS_HIP(launch_dot_rz32((const float*)B.x[1], p->r, N, p->partial, p->sc + kScRZNew, p->stream));
  return Status::ok();
}

}  // namespace

// With VPS_FLAG_GRAPHS the preconditioner (~20 kernels per level, fixed arguments) is captured once
// per solve mode into a HIP graph (fills are kernels, there are no memset nodes) and replayed;
// where capture is not possible the kernels are launched directly.
Status precondition(Problem* p, int mode) {
  if (!p->use_graphs || p->graph_failed[mode]) return precondition_launch(p, mode);
  if (!p->graph_stream) {
    if (hipStreamCreateWithFlags(&p->graph_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->graph_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->graph_out, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      p->use_graphs = false;
      return precondition_launch(p, mode);
    }
  }
  if (!p->precond_graph[mode]) {
    // capture on the private stream: every launch of precondition_launch goes to p->stream
    hipStream_t caller = p->stream;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->graph_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      p->graph_failed[mode] = true;
      return precondition_launch(p, mode);
    }
    p->stream = p->graph_stream;
    const Status s = precondition_launch(p, mode);
    p->stream = caller;
    hipError_t e = hipStreamEndCapture(p->graph_stream, &g);
    if (s.code == 0 && e == hipSuccess && g) e = hipGraphInstantiate(&p->precond_graph[mode], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (s.code) return s;
    if (e != hipSuccess || !p->precond_graph[mode]) {
      (void)hipGetLastError();
      p->precond_graph[mode] = nullptr;
      p->graph_failed[mode] = true;
      return precondition_launch(p, mode);
    }
  }
  VPS_HIP(hipEventRecord(p->graph_in, p->stream));
  VPS_HIP(hipStreamWaitEvent(p->graph_stream, p->graph_in, 0));
  VPS_HIP(hipGraphLaunch(p->precond_graph[mode], p->graph_stream));
  VPS_HIP(hipEventRecord(p->graph_out, p->graph_stream));
  VPS_HIP(hipStreamWaitEvent(p->stream, p->graph_out, 0));
  return Status::ok();
}

Status precondition_group(Problem* const* ps, int n, int mode) {
  const int prec = mode == 0 ? 0 : 1;
  std::vector<const void*> bs(n);
  std::vector<void*> xs(n);
  for (int i = 0; i < n; ++i) {
    Problem* p = ps[i];
    const long long N = p->lv[p->L].N;
    // x = 0 on entry without a fill: the first colour pass of the group's V-cycle (from zero)
    // writes every node
    if (mode == 0) {
      bs[i] = p->r;
      xs[i] = p->z;
    } else {
      LevelBuffers& B = p->lv[p->L];
      bs[i] = B.b[1];
      xs[i] = B.x[1];
    }
  }
  VPS_TRY(vcycle_group(ps, n, prec, bs.data(), xs.data(), true));
  for (int i = 0; i < n; ++i) {
    Problem* p = ps[i];
    const long long N = p->lv[p->L].N;
    if (mode == 0)
      VPS_HIP(launch_dot2(p->r, p->z, nullptr, nullptr, N, p->partial, p->sc + kScRZNew, p->stream));
    else
      VPS_HIP(launch_dot_rz32((const float*)p->lv[p->L].x[1], p->r, N, p->partial, p->sc + kScRZNew,
                               p->stream));
  }
  return Status::ok();
}

Status pcg_begin_launch(Problem* p, int mode, const double* b, double* x, CgState* cs) {
  if (!p->r) return Status{-1, "problem was created without solver vectors"};
  if (!p->has(mode == 0 ? 0 : 1)) return Status{-1, "solve mode needs the matching hierarchy flag"};
  const long long N = p->lv[p->L].N;
  *cs = CgState();
  VPS_HIP(hipMemsetAsync(p->bad, 0, sizeof(int), p->stream));
  // r = b (interior), x = 0 and, mixed, the FP32 copy of r (the FP32 V-cycle's input) in one pass
  VPS_HIP(launch_copy_interior_norm(p->dim, p->lv[p->L].g.n1d, b, p->r, p->partial, p->sc + kScBB, p->bad, p->stream,
                                    mode == 1 ? static_cast<float*>(p->lv[p->L].b[1]) : nullptr, x));
  VPS_HIP(hipMemcpyAsync(p->host_sc, p->sc, kScCount * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  VPS_HIP(hipMemcpyAsync(p->host_bad, p->bad, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  return Status::ok();
}

Status pcg_begin_check(Problem* p, CgState* cs) {
  cs->bb = p->host_sc[kScBB];
  if (*p->host_bad || !std::isfinite(cs->bb)) {
    cs->done = true;
    cs->stats.status = -6;
  } else if (cs->bb == 0.0) {
    cs->done = true;
    cs->stats.rel_residual = 0.0;
  }
  return Status::ok();
}

Status pcg_begin_after_precond(Problem* p, int mode) {
  const long long N = p->lv[p->L].N;
  VPS_HIP(launch_cg_beta(p->sc, 0, p->stream));  // rz <- rz_new (beta unused here)
  if (mode == 1)
    VPS_HIP(launch_cast(1, cg_z32(p, mode), p->p, N, p->stream));  // p = z, widened exactly
  else
    VPS_HIP(hipMemcpyAsync(p->p, p->z, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  return Status::ok();
}

Status pcg_begin(Problem* p, int mode, const double* b, double* x, CgState* cs) {
  VPS_TRY(pcg_begin_launch(p, mode, b, x, cs));
  VPS_HIP(hipStreamSynchronize(p->stream));
  VPS_TRY(pcg_begin_check(p, cs));
  if (cs->done) return Status::ok();
  VPS_TRY(precondition(p, mode));
  return pcg_begin_after_precond(p, mode);
}

Status pcg_iterate_launch(Problem* p, int mode, double* x, CgState* cs) {
  (void)mode;
  const long long N = p->lv[p->L].N;
  bool fused = false;
  VPS_HIP(launch_operator_pq(p->geom(p->L), p->p, p->q, p->partial, p->n_partial, p->sc + kScPQ, p->stream,
                             &fused));
  if (!fused) {
    VPS_HIP(launch_operator(p->geom(p->L), 0, p->p, nullptr, p->q, p->stream));
    VPS_HIP(launch_dot2(p->p, p->q, nullptr, nullptr, N, p->partial, p->sc + kScPQ, p->stream));
  }
  float* r32 = mode == 1 ? static_cast<float*>(p->lv[p->L].b[1]) : nullptr;  // input of the FP32 V-cycle
  VPS_HIP(launch_cg_update(x, p->r, p->p, p->q, p->z, cg_z32(p, mode), N, p->sc, p->partial, r32, p->stream));
  VPS_HIP(hipMemcpyAsync(p->host_sc, p->sc, kScCount * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  (void)cs;
  return Status::ok();
}

Status pcg_decide(Problem* p, int mode, double rtol, int maxit, CgState* cs) {
  (void)mode;
  const double pq = p->host_sc[kScPQ], rz = p->host_sc[kScRZ], rr = p->host_sc[kScRR];
  cs->it += 1;
  cs->stats.iterations = cs->it;
  if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rz) || !std::isfinite(rr)) {
    cs->done = true;
    cs->stats.status = -5;
    return Status::ok();
  }
  cs->rel = std::sqrt(rr / cs->bb);
  cs->stats.rel_residual = cs->rel;
  if (cs->rel <= rtol) {
    cs->done = true;
    cs->stats.status = 0;
  } else if (cs->it >= maxit) {
    cs->done = true;
    cs->stats.status = -4;
  }
  return Status::ok();
}

Status pcg_after_precond(Problem* p, int mode) {
  const long long N = p->lv[p->L].N;
  // flexible (Polak-Ribiere) beta whenever the preconditioner is not symmetric: FP32 V-cycle
  // (rounding) or the literal colour order after the coarse correction
  VPS_HIP(launch_cg_beta(p->sc, (mode == 1 || p->post_same_order) ? 1 : 0, p->stream));
  VPS_HIP(launch_cg_direction(p->p, p->z, cg_z32(p, mode), N, p->sc, p->stream));
  return Status::ok();
}

Status pcg_iterate_finish(Problem* p, int mode, double rtol, int maxit, CgState* cs) {
  VPS_TRY(pcg_decide(p, mode, rtol, maxit, cs));
  if (cs->done) return Status::ok();
  VPS_TRY(precondition(p, mode));
  return pcg_after_precond(p, mode);
}

Status pcg_end_launch(Problem* p, const double* b, const double* x, const CgState* cs, bool* pending) {
  *pending = false;
  if (cs->stats.status == -6 || cs->bb == 0.0) return Status::ok();
  const long long N = p->lv[p->L].N;
  // |b - A x|^2 in one pass where a fused operator form serves the level, else through q
  bool fused = false;
  VPS_HIP(launch_residual_norm2(p->geom(p->L), x, b, p->partial, p->n_partial, p->sc + kScTrue, p->stream,
                                &fused));
  if (!fused) {
    VPS_HIP(launch_operator(p->geom(p->L), 0, x, b, p->q, p->stream));  // q = b - A x (interior)
    VPS_HIP(launch_dot2(p->q, p->q, nullptr, nullptr, N, p->partial, p->sc + kScTrue, p->stream));
  }
  VPS_HIP(hipMemcpyAsync(p->host_sc, p->sc, kScCount * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  *pending = true;
  return Status::ok();
}

void pcg_end_finish(const Problem* p, CgState* cs) {
  cs->stats.true_rel_residual = std::sqrt(p->host_sc[kScTrue] / cs->bb);
}

Status pcg_end(Problem* p, const double* b, double* x, CgState* cs) {
  bool pending = false;
  VPS_TRY(pcg_end_launch(p, b, x, cs, &pending));
  if (!pending) return Status::ok();
  VPS_HIP(hipStreamSynchronize(p->stream));
  pcg_end_finish(p, cs);
  return Status::ok();
}

Status pcg(Problem* p, int mode, const double* b, double* x, double rtol, int maxit, SolveStats* out) {
  CgState cs;
  VPS_TRY(pcg_begin(p, mode, b, x, &cs));
  while (!cs.done) {
    VPS_TRY(pcg_iterate_launch(p, mode, x, &cs));
    VPS_HIP(hipStreamSynchronize(p->stream));
    VPS_TRY(pcg_iterate_finish(p, mode, rtol, maxit, &cs));
  }
  VPS_TRY(pcg_end(p, b, x, &cs));
  if (out) *out = cs.stats;
  return Status::ok();
}

}  // namespace vps
