// extern "C" boundary of the library (declared in include/vps.h).  Validates
// arguments on the host, maps every failure to a status code plus a
// thread-local message, and never lets a C++ exception cross the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "vps.h"
#include "kernels.hpp"
#include "problem.hpp"
#include "tables.hpp"

struct vps_problem {
  vps::Problem* impl;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int from(const vps::Status& s) {
  if (s.code != 0) g_err = s.msg;
  return s.code;
}

bool valid_shape(int dim, int degree, int level, std::string* why) {
  if (dim != 2 && dim != 3) return *why = "dim must be 2 or 3", false;
  if (degree < 1 || degree > vps::kMaxDegree) return *why = "degree must be in 1..7", false;
  if (level < 1 || level > 20) return *why = "level must be in 1..20", false;
  const double n1d = (double)degree * std::ldexp(1.0, level) + 1.0;
  if (std::pow(n1d, dim) >= std::ldexp(1.0, 40)) return *why = "problem too large (N >= 2^40)", false;
  return true;
}

int check_level(const vps_problem* p, int level, int lo) {
  if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
  if (level < lo || level > p->impl->L)
    return fail(VPS_EINVAL, "level " + std::to_string(level) + " outside " + std::to_string(lo) + ".." +
                                std::to_string(p->impl->L));
  return VPS_OK;
}

int check_prec(int prec) { return (prec == 0 || prec == 1) ? VPS_OK : fail(VPS_EINVAL, "prec must be VPS_FP64 or VPS_FP32"); }

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    return fail(VPS_EINVAL, std::string("exception: ") + e.what());
  } catch (...) {
    return fail(VPS_EINVAL, "unknown exception");
  }
}

}  // namespace

namespace vps {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace vps

extern "C" {

const char* vps_last_error(void) { return g_err.c_str(); }

int vps_footprint_bytes(int dim, int degree, int fine_level, unsigned flags, size_t* bytes) {
  return guarded([&]() -> int {
    std::string why;
    if (!valid_shape(dim, degree, fine_level, &why)) return fail(VPS_EINVAL, why);
    if (!bytes) return fail(VPS_EINVAL, "null output");
    *bytes = vps::footprint_bytes(dim, degree, fine_level, flags);
    return VPS_OK;
  });
}

int vps_create(int dim, int degree, int fine_level, unsigned flags, void* hip_stream, vps_problem** out) {
  return guarded([&]() -> int {
    std::string why;
    if (!valid_shape(dim, degree, fine_level, &why)) return fail(VPS_EINVAL, why);
    if (!out) return fail(VPS_EINVAL, "null output");
    if (!(flags & (VPS_FLAG_FP64_HIERARCHY | VPS_FLAG_FP32_HIERARCHY)))
      flags |= VPS_FLAG_FP64_HIERARCHY;
    vps::Problem* impl = nullptr;
    vps::Status s = vps::create_problem(dim, degree, fine_level, flags, (hipStream_t)hip_stream, &impl);
    if (s.code) return from(s);
    *out = new vps_problem{impl};
    return VPS_OK;
  });
}

int vps_destroy(vps_problem* p) {
  return guarded([&]() -> int {
    if (!p) return VPS_OK;
    delete p->impl;
    delete p;
    return VPS_OK;
  });
}

int vps_level_info(const vps_problem* p, int level, vps_level_info_t* out) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (!out) return fail(VPS_EINVAL, "null output");
    const vps::Problem& P = *p->impl;
    const vps::LevelGeom& g = P.geom(level);
    std::memset(out, 0, sizeof(*out));
    out->dim = P.dim;
    out->degree = P.k;
    out->level = level;
    out->n1d = g.n1d;
    out->n_dofs = P.lv[level].N;
    long long inner = g.n1d - 2, cells = g.ncells, verts = g.ncells - 1;
    out->n_interior = P.dim == 2 ? inner * inner : inner * inner * inner;
    out->n_cells = P.dim == 2 ? cells * cells : cells * cells * cells;
    out->n_patches = P.dim == 2 ? verts * verts : verts * verts * verts;
    out->n_colors = 1 << P.dim;
    for (int c = 0; c < out->n_colors; ++c) {
      long long cnt = 1;
      for (int a = 0; a < P.dim; ++a) cnt *= g.ncells / 2 - ((c >> a) & 1);
      out->color_count[c] = cnt;
    }
    out->h = g.h;
    return VPS_OK;
  });
}

int vps_dof_index(const vps_problem* p, int level, const int* coords, long long* idx) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (!coords || !idx) return fail(VPS_EINVAL, "null argument");
    const vps::LevelGeom& g = p->impl->geom(level);
    long long v = 0;
    for (int a = p->impl->dim - 1; a >= 0; --a) {
      if (coords[a] < 0 || coords[a] >= g.n1d) return fail(VPS_EINVAL, "coordinate out of range");
      v = v * g.n1d + coords[a];
    }
    *idx = v;
    return VPS_OK;
  });
}

int vps_patch_first_index(const vps_problem* p, int level, int color, long long* out, long long cap, long long* n) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    const int dim = p->impl->dim, k = p->impl->k;
    if (color < 0 || color >= (1 << dim)) return fail(VPS_EINVAL, "color out of range");
    if (!n) return fail(VPS_EINVAL, "null count");
    const vps::LevelGeom& g = p->impl->geom(level);
    long long cnt[3] = {1, 1, 1};
    int par[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      par[a] = (color >> a) & 1;
      cnt[a] = g.ncells / 2 - par[a];
      if (cnt[a] < 0) cnt[a] = 0;
    }
    const long long total = cnt[0] * cnt[1] * cnt[2];
    *n = total;
    if (!out || cap < total) return VPS_OK;
    long long i = 0;
    for (long long t2 = 0; t2 < cnt[2]; ++t2)
      for (long long t1 = 0; t1 < cnt[1]; ++t1)
        for (long long t0 = 0; t0 < cnt[0]; ++t0) {
          const long long s0 = k * (par[0] + 2 * t0), s1 = k * (par[1] + 2 * t1), s2 = k * (par[2] + 2 * t2);
          out[i++] = dim == 2 ? s1 * g.n1d + s0 : (s2 * g.n1d + s1) * g.n1d + s0;
        }
    return VPS_OK;
  });
}

int vps_operator_apply(vps_problem* p, int level, int prec, const void* x, void* y) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (int e = check_prec(prec)) return e;
    if (!x || !y) return fail(VPS_EINVAL, "null vector");
    const vps::LevelGeom& g = p->impl->geom(level);
    hipError_t e = vps::launch_operator(g, prec, x, nullptr, y, p->impl->stream);
    if (e == hipSuccess) e = vps::launch_zero_boundary(g, prec, y, p->impl->stream);
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("operator launch: ") + hipGetErrorString(e));
  });
}

int vps_residual(vps_problem* p, int level, int prec, const void* b, const void* x, void* r) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (int e = check_prec(prec)) return e;
    if (!b || !x || !r) return fail(VPS_EINVAL, "null vector");
    const vps::LevelGeom& g = p->impl->geom(level);
    hipError_t e = vps::launch_operator(g, prec, x, b, r, p->impl->stream);
    if (e == hipSuccess) e = vps::launch_zero_boundary(g, prec, r, p->impl->stream);
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("residual launch: ") + hipGetErrorString(e));
  });
}

int vps_smoother_apply(vps_problem* p, int level, int prec, int mode, int reverse_colors, const void* b, void* x) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (int e = check_prec(prec)) return e;
    if (mode != VPS_MULTIPLICATIVE && mode != VPS_ADDITIVE && mode != VPS_MULTIPLICATIVE_BOUNDARY &&
        mode != VPS_MULTIPLICATIVE_SEPARATE && mode != VPS_MULTIPLICATIVE_MFMA)
      return fail(VPS_EINVAL, "bad smoother mode");
    if (!b || !x) return fail(VPS_EINVAL, "null vector");
    return from(vps::smoother(p->impl, level, prec, mode, reverse_colors != 0, b, x));
  });
}

int vps_color_pass(vps_problem* p, int level, int prec, int mode, int color, const void* b, void* x) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (int e = check_prec(prec)) return e;
    if (mode != VPS_MULTIPLICATIVE && mode != VPS_ADDITIVE && mode != VPS_MULTIPLICATIVE_BOUNDARY &&
        mode != VPS_MULTIPLICATIVE_SEPARATE && mode != VPS_MULTIPLICATIVE_MFMA)
      return fail(VPS_EINVAL, "bad smoother mode");
    if (color < 0 || color >= (1 << p->impl->dim)) return fail(VPS_EINVAL, "color out of range");
    if (!b || !x) return fail(VPS_EINVAL, "null vector");
    return from(vps::colour_pass(p->impl, level, prec, mode, color, b, x));
  });
}

int vps_launch_geometry_check(int dim, int degree, int fine_level, long long* blocks_checked) {
  return guarded([&]() -> int {
    std::string why;
    if (!valid_shape(dim, degree, fine_level, &why)) return fail(VPS_EINVAL, why);
    long long blocks = 0;
    for (int lvl = 1; lvl <= fine_level; ++lvl) {
      const vps::LevelGeom g = vps::make_geom(dim, degree, lvl);
      if (!vps::check_colour_launches(g, &blocks, &why) || !vps::check_grid_launches(g, &why))
        return fail(VPS_EINVAL, "level " + std::to_string(lvl) + ": " + why);
    }
    if (blocks_checked) *blocks_checked = blocks;
    return VPS_OK;
  });
}

int vps_restrict_noalloc(int dim, int degree, int fine_level, int prec, const void* r_fine, void* r_coarse,
                         void* hip_stream) {
  return guarded([&]() -> int {
    std::string why;
    if (!valid_shape(dim, degree, fine_level, &why)) return fail(VPS_EINVAL, why);
    if (fine_level < 2) return fail(VPS_EINVAL, "restriction needs fine_level >= 2");
    if (int e = check_prec(prec)) return e;
    const size_t need = (size_t)vps::restrict_scratch_elems(dim, degree, fine_level) * (prec == 0 ? 8 : 4);
    if (need > vps::noalloc_scratch_bytes())
      return fail(VPS_EINVAL, "restriction scratch of " + std::to_string(need) + " bytes exceeds the " +
                                  std::to_string(vps::noalloc_scratch_bytes()) +
                                  " bytes of the allocation-free entry point (use vps_restrict)");
    if (!r_fine || !r_coarse) return fail(VPS_EINVAL, "null vector");
    void* t = nullptr;
    hipError_t e = vps::noalloc_scratch(&t);
    if (e != hipSuccess) return fail(VPS_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    e = vps::launch_restrict(vps::make_geom(dim, degree, fine_level), prec, r_fine, r_coarse, t,
                             static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("restrict launch: ") + hipGetErrorString(e));
  });
}

int vps_restrict(vps_problem* p, int fine_level, int prec, const void* r_fine, void* r_coarse) {
  return guarded([&]() -> int {
    if (int e = check_level(p, fine_level, 2)) return e;
    if (int e = check_prec(prec)) return e;
    if (!r_fine || !r_coarse) return fail(VPS_EINVAL, "null vector");
    const vps::LevelBuffers& B = p->impl->lv[fine_level];
    if (!B.r[prec]) return fail(VPS_EINVAL, "restriction in this precision needs the matching hierarchy flag");
    hipError_t e = vps::launch_restrict(p->impl->geom(fine_level), prec, r_fine, r_coarse, B.t[prec],
                                        p->impl->stream);
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("restrict launch: ") + hipGetErrorString(e));
  });
}

int vps_prolongate_add(vps_problem* p, int fine_level, int prec, const void* e_coarse, void* x_fine) {
  return guarded([&]() -> int {
    if (int e = check_level(p, fine_level, 2)) return e;
    if (int e = check_prec(prec)) return e;
    if (!e_coarse || !x_fine) return fail(VPS_EINVAL, "null vector");
    hipError_t e = vps::launch_prolongate_add(p->impl->geom(fine_level), prec, e_coarse, x_fine, p->impl->stream);
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("prolongate launch: ") + hipGetErrorString(e));
  });
}

int vps_coarse_solve(vps_problem* p, int prec, const void* b, void* x) {
  return guarded([&]() -> int {
    if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
    if (int e = check_prec(prec)) return e;
    if (!b || !x) return fail(VPS_EINVAL, "null vector");
    return from(vps::coarse_solve(p->impl, prec, b, x));
  });
}

int vps_vcycle(vps_problem* p, int prec, const void* b, void* x) {
  return guarded([&]() -> int {
    if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
    if (int e = check_prec(prec)) return e;
    if (!b || !x) return fail(VPS_EINVAL, "null vector");
    return from(vps::vcycle(p->impl, prec, b, x));
  });
}

int vps_pcg_solve(vps_problem* p, int solve_mode, const double* b, double* x, double rtol, int maxit,
                  vps_solve_stats_t* stats) {
  return guarded([&]() -> int {
    if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
    if (solve_mode != VPS_SOLVE_FP64 && solve_mode != VPS_SOLVE_MIXED) return fail(VPS_EINVAL, "bad solve mode");
    if (!b || !x) return fail(VPS_EINVAL, "null vector");
    if (!(rtol > 0.0) || maxit < 1) return fail(VPS_EINVAL, "rtol must be > 0 and maxit >= 1");
    vps::SolveStats st;
    vps::Status s = vps::pcg(p->impl, solve_mode, b, x, rtol, maxit, &st);
    if (s.code) return from(s);
    if (stats) {
      stats->iterations = st.iterations;
      stats->rel_residual = st.rel_residual;
      stats->true_rel_residual = st.true_rel_residual;
      stats->status = st.status;
    }
    if (st.status != 0)
      return fail(st.status, st.status == VPS_ENOCONV      ? "iteration limit reached"
                             : st.status == VPS_EBREAKDOWN ? "CG breakdown (p.Ap <= 0 or non-finite scalar)"
                                                           : "non-finite right-hand side");
    return VPS_OK;
  });
}

int vps_fmg_solve(vps_problem* p, int prec, const void* const* b_levels, void* x, double eps, int maxit,
                  vps_solve_stats_t* stats) {
  return guarded([&]() -> int {
    if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
    if (int e = check_prec(prec)) return e;
    if (!b_levels || !x) return fail(VPS_EINVAL, "null vector");
    for (int l = 0; l < p->impl->L; ++l)
      if (!b_levels[l]) return fail(VPS_EINVAL, "null right-hand side on a level");
    if (!(eps > 0.0) || maxit < 0) return fail(VPS_EINVAL, "eps must be > 0 and maxit >= 0");
    vps::SolveStats st;
    vps::Status s = vps::fmg(p->impl, prec, b_levels, x, eps, maxit, &st);
    if (s.code) return from(s);
    if (stats) {
      stats->iterations = st.iterations;
      stats->rel_residual = st.rel_residual;
      stats->true_rel_residual = st.true_rel_residual;
      stats->status = st.status;
    }
    if (st.status != 0)
      return fail(st.status, st.status == VPS_ENOCONV ? "V-cycle limit reached" : "non-finite right-hand side or residual");
    return VPS_OK;
  });
}

int vps_rhs_sine_modes(vps_problem* p, int level, int prec, int n_modes, const int* kappa, const double* coef,
                       void* b) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (int e = check_prec(prec)) return e;
    if (n_modes < 0 || (n_modes > 0 && (!kappa || !coef)) || !b) return fail(VPS_EINVAL, "bad mode arrays");
    const vps::Problem& P = *p->impl;
    const vps::LevelGeom& g = P.geom(level);
    const vps::Tables1D& t = vps::tables_for_degree(P.k);
    const int k = P.k, np = k + 1;
    const double pi = std::acos(-1.0);
    // 1D load vectors g[i] = int sin(pi kappa x) phi_i(x) dx, (k+1)-point Gauss per cell
    std::vector<double> V(np * np);  // V[i*np + q] = phi_i(x_q)
    for (int i = 0; i < np; ++i)
      for (int q = 0; q < np; ++q) V[i * np + q] = vps::lagrange(t.gll, i, t.gauss_x[q]);
    std::vector<double> G((size_t)std::max(n_modes, 1) * P.dim * g.n1d, 0.0);
    for (int m = 0; m < n_modes; ++m)
      for (int a = 0; a < P.dim; ++a) {
        double* gv = &G[((size_t)m * P.dim + a) * g.n1d];
        const double kap = kappa[m * P.dim + a];
        for (long long c = 0; c < g.ncells; ++c)
          for (int q = 0; q < np; ++q) {
            const double xq = (c + t.gauss_x[q]) * g.h;
            const double f = t.gauss_w[q] * g.h * std::sin(pi * kap * xq);
            for (int i = 0; i < np; ++i) gv[c * k + i] += V[i * np + q] * f;
          }
      }
    double *dG = nullptr, *dc = nullptr;
    auto cleanup = [&] {
      if (dG) (void)hipFree(dG);
      if (dc) (void)hipFree(dc);
    };
    if (hipMalloc(&dG, G.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&dc, (size_t)std::max(n_modes, 1) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      cleanup();
      return fail(VPS_ENOMEM, "rhs scratch allocation failed");
    }
    hipError_t e = hipMemcpyAsync(dG, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess && n_modes > 0)
      e = hipMemcpyAsync(dc, coef, n_modes * sizeof(double), hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess) e = vps::launch_rhs_separable(g, prec, n_modes, dG, dc, b, P.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
    cleanup();
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("rhs: ") + hipGetErrorString(e));
  });
}

int vps_l2_error_sine_modes(vps_problem* p, int level, int n_modes, const int* kappa, const double* ucoef, int nq,
                            const double* x, double* err) {
  return guarded([&]() -> int {
    if (int e = check_level(p, level, 1)) return e;
    if (n_modes < 0 || (n_modes > 0 && (!kappa || !ucoef)) || !x || !err) return fail(VPS_EINVAL, "bad arguments");
    const vps::Problem& P = *p->impl;
    const int k = P.k, np = k + 1;
    if (nq == 0) nq = np;
    if (nq < 1 || nq > 16) return fail(VPS_EINVAL, "nq must be 0 (k+1) or in 1..16");
    const vps::LevelGeom& g = P.geom(level);
    const vps::Tables1D& t = vps::tables_for_degree(k);
    const double pi = std::acos(-1.0);
    std::vector<double> xq, wq;
    vps::gauss_legendre(nq, xq, wq);
    std::vector<double> V((size_t)nq * np);  // V[q*np + i] = phi_i(xq_q)
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < np; ++i) V[(size_t)q * np + i] = vps::lagrange(t.gll, i, xq[q]);
    const size_t na = (size_t)g.ncells * nq;
    std::vector<double> S((size_t)std::max(n_modes, 1) * P.dim * na, 0.0);
    for (int m = 0; m < n_modes; ++m)
      for (int a = 0; a < P.dim; ++a) {
        const double kap = kappa[m * P.dim + a];
        double* sv = &S[((size_t)m * P.dim + a) * na];
        for (long long c = 0; c < g.ncells; ++c)
          for (int q = 0; q < nq; ++q) sv[c * nq + q] = std::sin(pi * kap * (c + xq[q]) * g.h);
      }
    const int nparts = 4096;
    const size_t bytes[5] = {V.size() * 8, wq.size() * 8, S.size() * 8, (size_t)std::max(n_modes, 1) * 8,
                             (size_t)nparts * 8};
    void* d[5] = {};
    auto cleanup = [&] {
      for (void* q : d)
        if (q) (void)hipFree(q);
    };
    for (int i = 0; i < 5; ++i)
      if (hipMalloc(&d[i], bytes[i]) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(VPS_ENOMEM, "L2 error scratch allocation failed");
      }
    hipError_t e = hipMemcpyAsync(d[0], V.data(), bytes[0], hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d[1], wq.data(), bytes[1], hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d[2], S.data(), bytes[2], hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess && n_modes > 0)
      e = hipMemcpyAsync(d[3], ucoef, (size_t)n_modes * 8, hipMemcpyHostToDevice, P.stream);
    if (e == hipSuccess)
      e = vps::launch_l2_error(g, x, (const double*)d[0], (const double*)d[1], (const double*)d[2],
                               (const double*)d[3], n_modes, nq, (double*)d[4], nparts, P.stream);
    std::vector<double> part(nparts);
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), d[4], bytes[4], hipMemcpyDeviceToHost, P.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
    cleanup();
    if (e != hipSuccess) return fail(VPS_EHIP, std::string("L2 error: ") + hipGetErrorString(e));
    double sum = 0.0;
    for (double v : part) sum += v;
    *err = std::sqrt(sum);
    return VPS_OK;
  });
}

int vps_synchronize(vps_problem* p) {
  return guarded([&]() -> int {
    if (!p || !p->impl) return fail(VPS_EINVAL, "null problem");
    hipError_t e = hipStreamSynchronize(p->impl->stream);
    return e == hipSuccess ? VPS_OK : fail(VPS_EHIP, std::string("synchronize: ") + hipGetErrorString(e));
  });
}

int vps_host_table(int k, int which, double* out, int cap, int* n) {
  return guarded([&]() -> int {
    if (k < 1 || k > vps::kMaxDegree) return fail(VPS_EINVAL, "degree out of range");
    if (!n) return fail(VPS_EINVAL, "null count");
    const vps::Tables1D& t = vps::tables_for_degree(k);
    const std::vector<double>* v = nullptr;
    switch (which) {
      case 0: v = &t.gll; break;
      case 1: v = &t.Ahat; break;
      case 2: v = &t.Mhat; break;
      case 3: v = &t.S; break;
      case 4: v = &t.lam; break;
      case 5: v = &t.P; break;
      default: return fail(VPS_EINVAL, "unknown table");
    }
    *n = (int)v->size();
    if (out && cap >= *n) std::memcpy(out, v->data(), v->size() * sizeof(double));
    return VPS_OK;
  });
}

}  // extern "C"
