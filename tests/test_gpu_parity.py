"""GPU parity: every C-ABI entry point against the FP64 oracle on the same seeded inputs.

Bars: FP64 results within 1e-12 relative (2-norm) of the oracle; FP32 kernels
within 1e-5; mixed-precision CG solutions within 1e-8 of the FP64 solution.
Sizes span several tiles/workgroups and ragged tails.  The launch shapes of the
workload sizes are compared element by element in test_gpu_fullsize.py, and the
solvers at those sizes in test_gpu_solves.py.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import mesh, multigrid, rhs, smoother, transfer

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402

F64 = torch.float64
F32 = torch.float32


def dev(a, dtype=F64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def case(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


_PROBLEMS = {}


def problem(d, k, L):
    key = (d, k, L)
    if key not in _PROBLEMS:
        _PROBLEMS[key] = vps.Problem(d, k, L)
    return _PROBLEMS[key]


OP_CASES = [(2, 1, 5), (2, 2, 4), (2, 3, 3), (2, 4, 3), (2, 5, 2), (2, 6, 2), (2, 7, 2),
            (3, 1, 3), (3, 2, 3), (3, 3, 3), (3, 4, 2), (3, 5, 2), (3, 6, 1), (3, 7, 2)]


@pytest.mark.parametrize("d,k,L", OP_CASES)
def test_operator_and_residual(d, k, L):
    case("operator", d, k, L)
    P = problem(d, k, L)
    x = synth.random_interior(d, k, L, 11)
    b = synth.random_interior(d, k, L, 12)
    xg = x.copy()
    xg[mesh.boundary_mask(d, k, L)] = 7.0  # boundary input must be ignored
    ref = mesh.apply_operator(d, k, L, x)
    y = P.operator_apply(dev(xg))
    assert rel(host(y), ref) <= 1e-12
    r = P.residual(dev(b), dev(xg))
    assert rel(host(r), b - ref) <= 1e-12
    y32 = P.operator_apply(dev(xg, F32))
    assert rel(host(y32), ref) <= 2e-6


@pytest.mark.parametrize("d,k,L", [(2, 1, 4), (2, 2, 3), (2, 3, 3), (2, 5, 2), (2, 7, 2),
                                   (3, 1, 3), (3, 2, 3), (3, 3, 2), (3, 4, 2), (3, 5, 2), (3, 7, 1)])
@pytest.mark.parametrize("mode", ["mult", "add"])
def test_colour_pass(d, k, L, mode):
    case("colour_pass", d, k, L, mode)
    P = problem(d, k, L)
    b = synth.random_interior(d, k, L, 21)
    x = synth.random_interior(d, k, L, 22)
    for c in range(2 ** d):
        xt = dev(x)
        if mode == "mult":
            P.color_pass(dev(b), xt, c, vps.VPS_MULTIPLICATIVE)
            ref = smoother.colour_pass(d, k, L, b, x, c)
        else:
            P.color_pass(dev(b), xt, c, vps.VPS_ADDITIVE)
            I = smoother._colour_index_arrays(d, k, L, c)
            ref = x.copy()
            if len(I):
                import scipy.linalg as sla
                ref[I] += sla.lu_solve(smoother._patch_lu(d, k, L), b[I].T).T
        assert rel(host(xt), ref) <= 1e-12, c


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (2, 4, 3), (3, 2, 3), (3, 4, 2), (3, 3, 3)])
def test_multiplicative_smoother_both_orders(d, k, L):
    case("smoother", d, k, L)
    P = problem(d, k, L)
    b = synth.random_interior(d, k, L, 31)
    x = synth.random_interior(d, k, L, 32)
    for rev in (False, True):
        xt = dev(x)
        P.smoother_apply(dev(b), xt, vps.VPS_MULTIPLICATIVE, rev)
        assert rel(host(xt), smoother.multiplicative(d, k, L, b, x, reverse=rev)) <= 1e-12
    xt = dev(x, F32)
    P.smoother_apply(dev(b, F32), xt, vps.VPS_MULTIPLICATIVE, False)
    assert rel(host(xt), smoother.multiplicative(d, k, L, b, x)) <= 1e-5


def test_additive_smoother_2d_q2_16x16_seed0():
    """2D Q2 on 16x16 cells, one additive application to a U[-1,1] residual (seed 0), FP64."""
    d, k, L = 2, 2, 4
    case("additive C1", d, k, L)
    P = problem(d, k, L)
    r = synth.random_interior(d, k, L, 0)
    y = P.new()
    P.smoother_apply(dev(r), y, vps.VPS_ADDITIVE)
    ref = smoother.additive(d, k, L, r)
    got = host(y)
    assert rel(got, ref) <= 1e-12
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,k,L", [(2, 1, 5), (2, 2, 4), (2, 3, 3), (2, 6, 3), (2, 7, 2),
                                   (3, 1, 4), (3, 2, 3), (3, 3, 3), (3, 4, 2), (3, 5, 2), (3, 7, 2)])
def test_transfer(d, k, L):
    case("transfer", d, k, L)
    P = problem(d, k, L)
    r = synth.random_interior(d, k, L, 41)
    e = synth.random_interior(d, k, L - 1, 42)
    x = synth.random_interior(d, k, L, 43)
    rg = r.copy()
    rg[mesh.boundary_mask(d, k, L)] = 9.0  # boundary input must be ignored
    rc = P.restrict(dev(rg))
    assert rel(host(rc), transfer.restrict(d, k, L, r)) <= 1e-12
    xt = dev(x)
    P.prolongate_add(dev(e), xt)
    assert rel(host(xt), x + transfer.prolongate(d, k, L, e)) <= 1e-12
    rc32 = P.restrict(dev(r, F32))
    assert rel(host(rc32), transfer.restrict(d, k, L, r)) <= 2e-6


@pytest.mark.parametrize("d,k", [(2, 1), (2, 4), (2, 7), (3, 1), (3, 3), (3, 7)])
def test_coarse_solve(d, k):
    case("coarse", d, k)
    P = problem(d, k, 2)
    b = synth.random_interior(d, k, 1, 51)
    ref = multigrid.coarse_solve(d, k, b)
    x = dev(np.zeros_like(b))
    P.coarse_solve(dev(b), x)
    assert rel(host(x), ref) <= 1e-12
    x32 = dev(np.zeros_like(b), F32)
    P.coarse_solve(dev(b, F32), x32)
    assert rel(host(x32), ref) <= 1e-6


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (2, 5, 3), (3, 2, 3), (3, 4, 2), (3, 3, 3)])
def test_vcycle(d, k, L):
    case("vcycle", d, k, L)
    P = problem(d, k, L)
    b = synth.random_interior(d, k, L, 61)
    x = synth.random_interior(d, k, L, 62)
    ref = multigrid.vcycle(d, k, L, b, x)
    xt = dev(x)
    P.vcycle(dev(b), xt)
    assert rel(host(xt), ref) <= 1e-12
    xt = dev(x, F32)
    P.vcycle(dev(b, F32), xt)
    assert rel(host(xt), ref) <= 1e-5


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (2, 3, 4), (3, 2, 3), (3, 3, 2)])
def test_rhs_sine_modes(d, k, L):
    case("rhs", d, k, L)
    P = problem(d, k, L)
    kap, co = synth.fourier_modes(d, seed=5)
    b = P.rhs_sine_modes(kap, co)
    assert rel(host(b), rhs.rhs_sine_modes(d, k, L, kap, co)) <= 1e-12


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (3, 2, 3), (3, 3, 3)])
def test_pcg_fp64_matches_oracle(d, k, L):
    case("pcg fp64", d, k, L)
    P = problem(d, k, L)
    kap, co = synth.manufactured_sine(d)
    b = rhs.rhs_sine_modes(d, k, L, kap, co)
    x_ref, it_ref, _ = multigrid.pcg(d, k, L, b, 1e-8)
    x, st = P.pcg_solve(dev(b), rtol=1e-8)
    assert st.status == 0
    assert st.iterations == it_ref
    assert rel(host(x), x_ref) <= 1e-12
    true = np.linalg.norm(b - mesh.apply_operator(d, k, L, host(x))) / np.linalg.norm(b)
    assert true <= 1.01e-8 and abs(true - st.true_rel_residual) <= 1e-3 * true


@pytest.mark.parametrize("d,k,L", [(2, 3, 4), (3, 2, 3), (3, 4, 2)])
def test_pcg_mixed_within_1e8_of_fp64(d, k, L):
    case("pcg mixed", d, k, L)
    P = problem(d, k, L)
    kap, co = synth.fourier_modes(d, seed=1)
    b = rhs.rhs_sine_modes(d, k, L, kap, co)
    x_ref, _, _ = multigrid.pcg(d, k, L, b, 1e-12)
    x, st = P.pcg_solve(dev(b), rtol=1e-10, mode=vps.VPS_SOLVE_MIXED)
    assert st.status == 0
    assert rel(host(x), x_ref) <= 1e-8


def test_kernels_deterministic_and_boundary_untouched():
    d, k, L = 3, 3, 3
    case("determinism", d, k, L)
    P = problem(d, k, L)
    b = dev(synth.random_interior(d, k, L, 71))
    x0 = synth.random_interior(d, k, L, 72)
    bm = mesh.boundary_mask(d, k, L)
    x0[bm] = 3.5
    outs = []
    for _ in range(2):
        xt = dev(x0)
        P.vcycle(b, xt)
        outs.append(host(xt))
    assert np.array_equal(outs[0], outs[1])
    assert np.all(outs[0][bm] == 3.5)


def test_pcg_error_paths():
    d, k, L = 2, 2, 3
    P = problem(d, k, L)
    b = synth.random_interior(d, k, L, 81)
    b[100] = np.nan
    with pytest.raises(vps.VpsError) as e:
        P.pcg_solve(dev(b))
    assert e.value.status == vps.VPS_ENOTFINITE
    b = synth.random_interior(d, k, L, 82)
    x, st = P.pcg_solve(dev(b), rtol=1e-14, maxit=1)
    assert st.status == vps.VPS_ENOCONV and st.iterations == 1
    x, st = P.pcg_solve(dev(np.zeros_like(b)))
    assert st.status == 0 and st.iterations == 0 and float(x.abs().max()) == 0.0


# ------------------------------------------------------------- workload sizes

def test_full_size_operator_3d_q4():
    d, k, L = 3, 4, 6
    case("C4 operator", d, k, L)
    P = problem(d, k, L)
    x = synth.random_interior(d, k, L, 94)
    assert rel(host(P.operator_apply(dev(x))), mesh.apply_operator(d, k, L, x)) <= 1e-12


def test_full_size_3d_q3_pcg_fp64():
    """3D Q3 on 32^3 cells, manufactured sine rhs, FP64 CG + V-cycle to 1e-8."""
    d, k, L = 3, 3, 5
    case("C2 pcg", d, k, L)
    P = problem(d, k, L)
    kap, co = synth.manufactured_sine(d)
    bt = P.rhs_sine_modes(kap, co)
    b = rhs.rhs_sine_modes(d, k, L, kap, co)
    assert rel(host(bt), b) <= 1e-12
    x, st = P.pcg_solve(bt, rtol=1e-8)
    assert st.status == 0 and st.iterations <= 10
    xh = host(x)
    assert np.linalg.norm(b - mesh.apply_operator(d, k, L, xh)) <= 1.01e-8 * np.linalg.norm(b)
    err = rhs.l2_error(d, k, L, xh, kap, rhs.exact_solution_coefs(kap, co))
    assert err < 2e-6  # order k+1 discretisation error at h = 1/32


def rounding_floor(d, k, L, x, b):
    """eps * || |A| |x| || / ||b||: the relative residual that FP64 rounding of A x alone can produce."""
    A1, M1 = mesh.global_1d_matrices(k, L)
    A1, M1 = abs(A1), abs(M1)
    n = mesh.n1d(k, L)
    X = np.abs(x).reshape((n,) * d)
    Y = np.zeros_like(X)
    for direction in range(d):
        T = X
        for a in range(d):
            T = mesh.apply_1d(A1 if a == direction else M1, T, a, d)
        Y += T
    return np.finfo(np.float64).eps * np.linalg.norm(Y) / np.linalg.norm(b)


@pytest.mark.parametrize("d,k,L,tol", [(2, 7, 9, 1e-10), (3, 4, 6, 1e-8)])
def test_full_size_mixed_vs_fp64(d, k, L, tol):
    case("mixed vs fp64", d, k, L)
    P = problem(d, k, L)
    if d == 2:
        kap, co = synth.manufactured_sine(d)
    else:
        kap, co = synth.fourier_modes(d, seed=1)
    bt = P.rhs_sine_modes(kap, co)
    x64, s64 = P.pcg_solve(bt, rtol=tol)
    x32, s32 = P.pcg_solve(bt, rtol=tol, mode=vps.VPS_SOLVE_MIXED)
    assert s64.status == 0 and s32.status == 0
    assert s64.iterations == s32.iterations
    a, c = host(x64), host(x32)
    assert rel(c, a) <= 1e-8
    b = host(bt)
    assert s64.rel_residual <= tol and s32.rel_residual <= tol
    for sol in (a, c):
        # the true residual is also bounded by what FP64 rounding of A x allows (about 1e-9 for 2D Q7 512^2)
        floor = rounding_floor(d, k, L, sol, b)
        true = np.linalg.norm(b - mesh.apply_operator(d, k, L, sol)) / np.linalg.norm(b)
        print("true residual %.3e, rounding floor %.3e" % (true, floor), flush=True)
        assert true <= 1.01 * tol + 10 * floor
