// Host-side state of one Poisson problem: the level hierarchy, device scratch
// and the solver drivers (V-cycle, CG).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device_common.hpp"

namespace vps {

struct Status {
  int code = 0;
  std::string msg;
  static Status ok() { return {}; }
};

struct LevelBuffers {
  LevelGeom g{};
  long long N = 0;                  // nodes on the level
  void* b[2] = {nullptr, nullptr};  // V-cycle right-hand side per precision (levels < L; FP32 also L)
  void* x[2] = {nullptr, nullptr};  // V-cycle iterate per precision
  void* r[2] = {nullptr, nullptr};  // residual per precision (every level)
  void* t[2] = {nullptr, nullptr};  // restriction scratch per precision (3D levels >= 2)
};

struct Problem {
  int dim = 0, k = 0, L = 0;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  std::vector<LevelBuffers> lv;  // index 0 unused, 1..L
  double* c64_b = nullptr;       // FP64 coarse pair used by the FP32 V-cycle
  double* c64_x = nullptr;
  // CG state
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* sc = nullptr;       // scalar block (kScCount doubles)
  double* partial = nullptr;  // n_partial doubles: the reductions' partial sums
  long long n_partial = 0;    // max(2 * reduction_parts(), fused_reduction_parts(finest level))
  int* bad = nullptr;
  double* host_sc = nullptr;  // pinned mirror of sc
  int* host_bad = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0;
  bool post_same_order = false;
  bool boundary_smoother = false;  // V-cycles smooth with the Boundary colour-pass kernel
  bool separate_smoother = false;  // V-cycles smooth in the Separate form (residual kernel + solve kernel)
  bool mfma_smoother = false;      // V-cycles smooth with the matrix-core form where it exists
  // CG preconditioner per solve mode, captured once as a HIP graph and replayed every iteration
  // (the caller's stream may be the null stream, which cannot be captured: the graph is captured
  // on and replayed from a private stream ordered against the caller's by events)
  bool use_graphs = false;
  hipGraphExec_t precond_graph[2] = {nullptr, nullptr};
  bool graph_failed[2] = {false, false};
  hipStream_t graph_stream = nullptr;
  hipEvent_t graph_in = nullptr, graph_out = nullptr;

  ~Problem();
  bool has(int prec) const;
  const LevelGeom& geom(int level) const { return lv[level].g; }
};

// Message returned by vps_last_error() on the calling thread.
void set_last_error(const std::string& msg);

LevelGeom make_geom(int dim, int k, int level);
long long level_nodes(int dim, int k, int level);
size_t footprint_bytes(int dim, int degree, int L, unsigned flags);

Status create_problem(int dim, int k, int L, unsigned flags, hipStream_t st, Problem** out);

// Device steps (asynchronous on p->stream).
// x_zero: x is 0 on entry (the first colour then runs the additive kernel, same values)
Status smoother(Problem* p, int level, int prec, int mode, bool reverse, const void* b, void* x, bool x_zero = false);
Status colour_pass(Problem* p, int level, int prec, int mode, int colour, const void* b, void* x);
Status coarse_solve(Problem* p, int prec, const void* b, void* x);
Status vcycle(Problem* p, int prec, const void* b, void* x);
// V-cycle with `top` as its finest level: b, x live on level `top`, levels below use the
// hierarchy's buffers (top < L leaves levels above untouched).  top_zero: x is 0 on entry.
Status vcycle_top(Problem* p, int prec, int top, const void* b, void* x, bool top_zero);
// V-cycles of n problems of the same (dim, degree), all on one stream, in lockstep: every colour
// pass of a level is one packed launch over the problems that have that level.  Each problem's
// arithmetic (and result) is exactly that of vcycle() on it alone.
Status vcycle_group(Problem* const* ps, int n, int prec, const void* const* bL, void* const* xL, bool top_zero);

struct SolveStats {
  int iterations = 0;
  double rel_residual = 0, true_rel_residual = 0;
  int status = 0;
};
Status pcg(Problem* p, int mode, const double* b, double* x, double rtol, int maxit, SolveStats* st);
// Full multigrid: b_levels[l-1] is the right-hand side on level l (l = 1..L), all in `prec`;
// x (level L, `prec`) receives the result.  st->iterations counts the V-cycles after the
// nested iteration; synchronises once per V-cycle on the finest level.
Status fmg(Problem* p, int prec, const void* const* b_levels, void* x, double eps, int maxit, SolveStats* st);

// Stepwise CG (used by the server): same arithmetic as pcg(), one iteration per call.
struct CgState {
  int it = 0;
  double bb = 0, rel = 1.0;
  bool done = false;
  SolveStats stats;
};
Status pcg_begin(Problem* p, int mode, const double* b, double* x, CgState* cs);
// pcg_begin in parts, for callers that synchronise several problems at once: the launches up to
// the copy of b.b to the host; after a synchronisation, the check of b (sets cs->done for a
// non-finite or zero rhs); after the first preconditioner application, p = z.
Status pcg_begin_launch(Problem* p, int mode, const double* b, double* x, CgState* cs);
Status pcg_begin_check(Problem* p, CgState* cs);
Status pcg_begin_after_precond(Problem* p, int mode);
Status pcg_iterate_launch(Problem* p, int mode, double* x, CgState* cs);   // enqueue one iteration up to the norm copy
Status pcg_iterate_finish(Problem* p, int mode, double rtol, int maxit, CgState* cs);  // after sync: decide, enqueue precond
// pcg_iterate_finish in parts, for callers that precondition several problems together:
Status pcg_decide(Problem* p, int mode, double rtol, int maxit, CgState* cs);  // after sync; no launches
Status pcg_after_precond(Problem* p, int mode);  // z and r.z are ready: beta, new direction
// z = M r and r.z with the CG vectors (FP64 V-cycle, or FP32 V-cycle on the FP32 copy of r that
// cg_update / pcg_begin wrote, widened back) for one problem / a group (same dim, degree)
Status precondition(Problem* p, int mode);
Status precondition_group(Problem* const* ps, int n, int mode);
Status pcg_end(Problem* p, const double* b, double* x, CgState* cs);
// pcg_end in parts: the true-residual launches (*pending = false when there is nothing to compute),
// and after a synchronisation the relative true residual.
Status pcg_end_launch(Problem* p, const double* b, const double* x, const CgState* cs, bool* pending);
void pcg_end_finish(const Problem* p, CgState* cs);

}  // namespace vps
