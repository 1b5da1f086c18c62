"""Solver parity with the oracle at the workloads' own sizes (Alg. 1 V-cycle inside CG, Sec. 4.2).

  * 3D Q3, 32^3 cells, FP64 CG to 1e-8: the iteration count equals the oracle's CG and
    the solution agrees to 1e-12 (relative 2-norm);
  * the literal colour order of Alg. 1 (VPS_FLAG_POST_SAME_ORDER) with the flexible
    coefficient, FP64 and mixed, against the oracle's flexible CG at small sizes;
  * 2D Q7 512^2 (to 1e-10) and 3D Q4 64^3 (to 1e-8), FP64 and mixed, both colour orders:
    the error of every solution against the exact discrete solution A^{-1} b from the
    oracle's direct solve, and mixed against FP64;
  * Table 7's degree-3 (769^3 nodes) and degree-7 (897^3) problems: right-hand side and
    residual entries on sampled nodes recomputed by the oracle, the true residual, and
    for degree 3 the L2 error against the oracle's h^4 extrapolation.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import direct, mesh, multigrid, rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402

F64 = torch.float64
BOTH = vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY


def case(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_c2_fp64_cg_matches_the_oracle_cg():
    """3D Q3, 32^3 cells (912,673 nodes), manufactured sine, FP64 CG + V-cycle to 1e-8."""
    d, k, L = 3, 3, 5
    case("C2 fp64 cg", d, k, L)
    b = rhs.rhs_sine_modes(d, k, L, *synth.manufactured_sine(d))
    x_ref, it_ref, hist = multigrid.pcg(d, k, L, b, 1e-8)
    P = vps.Problem(d, k, L)
    x, st = P.pcg_solve(dev(b), rtol=1e-8)
    xh = host(x)
    err = rel(xh, x_ref)
    exact = direct.exact_solve(d, k, L, b)
    print("  iterations %d (oracle %d), vs oracle CG %.2e, vs exact %.2e (oracle CG vs exact %.2e)"
          % (st.iterations, it_ref, err, rel(xh, exact), rel(x_ref, exact)), flush=True)
    assert st.status == 0 and st.iterations == it_ref
    assert err <= 1e-12
    P.close()


@pytest.mark.parametrize("d,k,L", [(2, 3, 4), (3, 2, 3), (3, 4, 2), (3, 3, 3)])
def test_literal_colour_order_flexible_cg_matches_the_oracle(d, k, L):
    """The configuration the benchmark times: Alg. 1 with the same colour order before and after
    the coarse correction, and the flexible (Polak-Ribiere) coefficient."""
    case("literal order cg", d, k, L)
    b = rhs.rhs_sine_modes(d, k, L, *synth.fourier_modes(d, seed=1))
    x_ref, it_ref, _ = multigrid.pcg(d, k, L, b, 1e-10, flexible=True, post_reverse=False)
    P = vps.Problem(d, k, L, BOTH | vps.VPS_FLAG_POST_SAME_ORDER)
    x, st = P.pcg_solve(dev(b), rtol=1e-10)
    assert st.status == 0 and st.iterations == it_ref
    assert rel(host(x), x_ref) <= 1e-12
    xm, sm = P.pcg_solve(dev(b), rtol=1e-10, mode=vps.VPS_SOLVE_MIXED)
    assert sm.status == 0
    assert rel(host(xm), x_ref) <= 1e-8
    P.close()


# C3 and C4 with the stopping tolerance of each workload.  Bars: the solution error against the
# exact discrete solution, for both precisions (the benchmark spec's bound for the mixed result, 1e-8),
# and mixed against FP64.
@pytest.mark.parametrize("order", ["reverse", "literal"])
@pytest.mark.parametrize("d,k,L,rtol", [(2, 7, 9, 1e-10), (3, 4, 6, 1e-8)])
def test_config_solves_against_the_exact_solution(d, k, L, rtol, order):
    case("config solve", d, k, L, rtol, order)
    if d == 2:
        kap, co = synth.manufactured_sine(d)
    else:
        kap, co = synth.fourier_modes(d, seed=1)
    b = rhs.rhs_sine_modes(d, k, L, kap, co)
    exact = direct.exact_solve(d, k, L, b)
    flags = BOTH | (vps.VPS_FLAG_POST_SAME_ORDER if order == "literal" else 0)
    P = vps.Problem(d, k, L, flags)
    bt = P.rhs_sine_modes(kap, co)
    assert np.max(np.abs(host(bt) - b)) <= 1e-13 * np.max(np.abs(b))
    x64, s64 = P.pcg_solve(bt, rtol=rtol)
    x32, s32 = P.pcg_solve(bt, rtol=rtol, mode=vps.VPS_SOLVE_MIXED)
    a, c = host(x64), host(x32)
    e64, e32, emx = rel(a, exact), rel(c, exact), rel(c, a)
    print("  iterations fp64 %d mixed %d; error vs exact: fp64 %.2e mixed %.2e; mixed vs fp64 %.2e"
          % (s64.iterations, s32.iterations, e64, e32, emx), flush=True)
    assert s64.status == 0 and s32.status == 0
    # Both runs stop on the same test.  With the literal colour order the preconditioner is not
    # symmetric, and at 2D Q7 512^2 its FP32 rounding leaves the mixed run's third residual just
    # above 1e-10 where the FP64 run's is below it: the counts may differ by that one iteration.
    if order == "reverse":
        assert s64.iterations == s32.iterations
    else:
        assert abs(s64.iterations - s32.iterations) <= 1
    assert e64 <= 1e-8 and e32 <= 1e-8 and emx <= 1e-8
    P.close()


# ------------------------------------------------------------------ Table 7, degrees 3 and 7

class _DeviceGather:
    """Index a device vector with host index arrays (for the oracle's row-by-row operator)."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, ids):
        return self.t[torch.as_tensor(np.asarray(ids), device=self.t.device)].double().cpu().numpy()


def _sample_coords(d, n, seed, count=48):
    rng = np.random.default_rng(seed)
    pts = [np.full(d, 1), np.full(d, n - 2), np.full(d, n // 2), np.array([1, n - 2, n // 3][:d]),
           np.array([0, n // 2, 5][:d])]
    pts += [rng.integers(0, n, size=d) for _ in range(count)]
    return np.array(pts, dtype=np.int64)


@pytest.fixture(scope="module")
def q3_error_extrapolation():
    """The oracle's L2 error of the degree-3 sine problem (exact discrete solutions at 16^3 and
    32^3 cells), carried to 256^3 cells with the rate the two levels show (about h^4)."""
    d, k = 3, 3
    kap, co = synth.manufactured_sine(d)
    uc = rhs.exact_solution_coefs(kap, co)
    e = {}
    for L in (4, 5):
        e[L] = rhs.l2_error(d, k, L, direct.exact_solve(d, k, L, rhs.rhs_sine_modes(d, k, L, kap, co)), kap, uc)
    assert abs(e[4] / e[5] - 16) < 0.5  # asymptotic order k + 1 = 4
    return e[5] * (e[5] / e[4]) ** 3


@pytest.mark.parametrize("mode", [vps.VPS_SOLVE_FP64, vps.VPS_SOLVE_MIXED])
@pytest.mark.parametrize("k,L", [(3, 8), (7, 7)])
def test_table7_full_size(k, L, mode, request):
    """Table 7 (degree 3: 454M DoFs; degree 7: 721M DoFs), manufactured sine, reduction 1e-9, the
    benchmark's configuration (literal colour order, flexible CG)."""
    d = 3
    case("table 7", d, k, L, "mixed" if mode else "fp64")
    kap, co = synth.manufactured_sine(d)
    n = mesh.n1d(k, L)
    P = vps.Problem(d, k, L, BOTH | vps.VPS_FLAG_POST_SAME_ORDER)
    b = P.rhs_sine_modes(kap, co)
    coords = _sample_coords(d, n, seed=7 + k)
    flat = coords[:, 0] + n * (coords[:, 1] + n * coords[:, 2])
    bs = rhs.rhs_sine_modes_at(d, k, L, kap, co, coords)
    bmax = float(b.abs().max())
    assert np.max(np.abs(_DeviceGather(b)[flat] - bs)) <= 1e-13 * bmax
    x, st = P.pcg_solve(b, rtol=1e-9, mode=mode)
    assert st.status == 0
    r = P.residual(b, x)
    true = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
    # residual entries on the sampled nodes: b_i - (A x)_i with the oracle's rows.  At convergence
    # the two terms cancel to about 1e-9 of |b_i|, so the difference of two correctly rounded
    # evaluations is set by the magnitudes summed, S_i = |b_i| + sum |products of (A x)_i|: each
    # side's error is at most gamma_n S_i with n = d (2k+1) + 2 the depth of the sum-factorised
    # row (u = 2^-53), and the bar is twice that.
    gx = _DeviceGather(x)
    rs = bs - mesh.operator_rows(d, k, L, coords, gx)
    mag = np.abs(bs) + mesh.operator_rows(d, k, L, coords, gx, absolute=True)
    nd = d * (2 * k + 1) + 2
    gamma = nd * 2.0 ** -53 / (1 - nd * 2.0 ** -53)
    e_rows = np.max(np.abs(_DeviceGather(r)[flat] - rs) / np.maximum(mag, 1e-300))
    print("  iterations %d, true residual %.3e (library %.3e), sampled residual rows vs oracle %.2e of "
          "the summed magnitudes (bar %.2e)" % (st.iterations, true, st.true_rel_residual, e_rows, 2 * gamma),
          flush=True)
    assert e_rows <= 2 * gamma
    assert true <= 2e-9 and abs(true - st.true_rel_residual) <= 1e-3 * true
    if k == 3:
        pred = request.getfixturevalue("q3_error_extrapolation")
        err = P.l2_error_sine_modes(x, kap, rhs.exact_solution_coefs(kap, co))
        print("  L2 error %.4e, oracle extrapolation %.4e" % (err, pred), flush=True)
        assert abs(err / pred - 1) < 0.1
    del b, x, r
    P.close()


def test_mfma_smoother_solve_at_3d_q4_64():
    """The mixed solve of 3D Q4 64^3 with VPS_FLAG_MFMA_SMOOTHER (the V-cycle's FP32 colour passes on
    the matrix cores) against the exact discrete solution, with the benchmark spec's bound for mixed
    precision, and against the vector-form solve."""
    d, k, L = 3, 4, 6
    case("mfma smoother solve", d, k, L)
    kap, co = synth.fourier_modes(d, seed=1)
    b = rhs.rhs_sine_modes(d, k, L, kap, co)
    exact = direct.exact_solve(d, k, L, b)
    P = vps.Problem(d, k, L, BOTH | vps.VPS_FLAG_POST_SAME_ORDER | vps.VPS_FLAG_MFMA_SMOOTHER)
    Q = vps.Problem(d, k, L, BOTH | vps.VPS_FLAG_POST_SAME_ORDER)
    bt = P.rhs_sine_modes(kap, co)
    xm, sm = P.pcg_solve(bt, rtol=1e-8, mode=vps.VPS_SOLVE_MIXED)
    xv, sv = Q.pcg_solve(bt, rtol=1e-8, mode=vps.VPS_SOLVE_MIXED)
    em, ev = rel(host(xm), exact), rel(host(xv), exact)
    print("  iterations mfma %d vector %d; error vs exact mfma %.2e vector %.2e" % (sm.iterations, sv.iterations, em, ev),
          flush=True)
    assert sm.status == 0 and abs(sm.iterations - sv.iterations) <= 1
    assert em <= 1e-8
    P.close()
    Q.close()
