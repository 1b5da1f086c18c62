"""GPU parity at the launch shapes the kernels take at full workload sizes.

The colour-pass kernel picks its patches-per-workgroup shape from the launch size
(small launches take a shorter "latency" shape), and the 3D operator switches to
its streaming form from 32 cells per axis.  The small-size parity tests reach only
the small shapes, so these tests run every shape used at a workload size against
the FP64 oracle, element by element:

  * colour passes: every colour of 3D Q4 64^3 cells and 2D Q7 512^2 cells, and for
    every other (dim, degree) a level where every colour launches the default shape;
    multiplicative, additive and Boundary modes, FP64 and FP32.  Every patch of the
    colour is compared (first and last patch per axis, the ragged last workgroup of a
    row, Dirichlet-adjacent patches), and every entry outside the colour's patch
    interiors must be unchanged bit for bit.  Boundary entries of x and b are NaN:
    the kernels must never read them;
  * operator apply and residual in the streaming form (3D, 32 cells and up, every
    degree; 3D Q4 64^3; 2D Q7 512^2), and the 2D tile form with several tiles per
    axis for every degree, ragged and exact, FP64 and FP32;
  * restriction and prolongation with several tiles per axis, ragged and exact.

Bars (max-abs error over the compared entries, relative to the max-abs reference
value): FP64 1e-12.  FP32: the kernel sees inputs rounded to FP32 and the oracle
gets the same rounded inputs in FP64, so only the kernel's own FP32 arithmetic
shows.  A patch update is a residual (sums of about 3(2k+1) products per 1D stage)
followed by a solve with condition number kappa(A_j) <= 68 (3D, k <= 5; 157 in 2D,
k = 7); its forward error is of order kappa(A_j) * u32 * (|b| + |Abar||x|)/|A_j^-1 r|,
u32 = 2^-24 = 6e-8.  The bars below are stated per case and leave a factor of at
least 4 over the errors measured on MI355X.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import mesh, smoother, transfer

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402

F64 = torch.float64
F32 = torch.float32
U32 = 2.0 ** -24


def case(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def as_seen(a, dtype):
    """The FP64 values a kernel of `dtype` receives."""
    return a.astype(np.float32).astype(np.float64) if dtype == F32 else np.array(a, dtype=np.float64)


def maxrel(got, ref):
    s = np.max(np.abs(ref))
    return np.max(np.abs(got - ref)) / (s if s > 0 else 1.0)


def poisoned(a, d, k, L):
    out = np.array(a, dtype=np.float64)
    out[mesh.boundary_mask(d, k, L)] = np.nan
    return out


_P = {}


def problem(d, k, L):
    key = (d, k, L)
    if key not in _P:
        for old in list(_P):
            _P.pop(old).close()
        _P[key] = vps.Problem(d, k, L)
    return _P[key]


# ------------------------------------------------------------------ colour passes

# (d, k, L): the two workload levels, then per (d, k) a level whose colours all launch the default
# shape (at least 1024 workgroups, or a degree whose small-launch shape is the default one).  3D Q3
# at 32^3 cells launches the default shape for colour 0 and the small shape for the others.
COLOUR_CASES = [(3, 4, 6), (2, 7, 9), (3, 3, 5), (3, 1, 7), (3, 2, 6), (3, 4, 5), (3, 5, 4), (3, 6, 4),
                (3, 7, 4), (2, 1, 10), (2, 2, 9), (2, 3, 9), (2, 4, 8), (2, 5, 8), (2, 6, 8)]
# FP32 bars per dimension (see the module docstring)
TOL32 = {2: 2e-5, 3: 1e-5}

MODES = [("mult", vps.VPS_MULTIPLICATIVE), ("add", vps.VPS_ADDITIVE), ("boundary", vps.VPS_MULTIPLICATIVE_BOUNDARY)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,L", COLOUR_CASES)
def test_colour_pass_every_patch(d, k, L, prec):
    dtype = F64 if prec == "fp64" else F32
    tol = 1e-12 if prec == "fp64" else TOL32[d]
    P = problem(d, k, L)
    b = as_seen(synth.random_interior(d, k, L, 101), dtype)
    x = as_seen(synth.random_interior(d, k, L, 102), dtype)
    bd = to_dev(poisoned(b, d, k, L), dtype)
    x_pois = poisoned(x, d, k, L)
    worst = {}
    for c in range(2 ** d):
        verts = mesh.patches_of_colour(d, L, c)
        C = mesh.patch_box_ids_many(d, k, L, verts, interior=False)
        I = mesh.patch_box_ids_many(d, k, L, verts, interior=True)
        ref_mult = smoother.patch_update_local_many(d, k, L, x[C], b[I])
        ref_add = x[I] + smoother.patch_solve_many(d, k, L, b[I])
        outside = np.ones(x.shape, dtype=bool)
        outside[I.reshape(-1)] = False
        for name, mode in MODES:
            case("colour pass", d, k, L, prec, name, "colour", c, "patches", len(verts))
            xt = to_dev(x_pois, dtype)
            P.color_pass(bd, xt, c, mode)
            got = host(xt)
            ref = ref_add if name == "add" else ref_mult
            e = maxrel(got[I], ref)
            worst[name] = max(worst.get(name, 0.0), e)
            assert e <= tol, (name, c, e)
            assert np.array_equal(got[outside], x_pois[outside], equal_nan=True), (name, c)
            del xt
    print("  max error / max |ref|:", {m: "%.2e" % v for m, v in worst.items()}, flush=True)


# ------------------------------------------------------------------ operator and residual

# 2D tiles hold (64, 13, 9, 8, 8, 8, 7) x (16, 8, 8, 6, 5, 4, 4) cells for K = 1..7: the 2D levels
# below give 2..8 tiles per axis, ragged along x0 for K = 2, 3, 7 and along x1 for K = 4, 5.
OP_CASES = [(3, 1, 5), (3, 2, 5), (3, 3, 5), (3, 4, 5), (3, 5, 5), (3, 6, 5), (3, 7, 5), (3, 4, 6), (2, 7, 9),
            (2, 1, 7), (2, 2, 6), (2, 3, 6), (2, 4, 5), (2, 5, 5), (2, 6, 5), (2, 7, 5)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,L", OP_CASES)
def test_operator_and_residual_streaming(d, k, L, prec):
    dtype = F64 if prec == "fp64" else F32
    tol = 1e-12 if prec == "fp64" else 3e-6
    case("operator", d, k, L, prec)
    P = problem(d, k, L)
    x = as_seen(synth.random_interior(d, k, L, 111), dtype)
    b = as_seen(synth.random_interior(d, k, L, 112), dtype)
    ax = mesh.apply_operator(d, k, L, x)
    xd = to_dev(poisoned(x, d, k, L), dtype)
    y = host(P.operator_apply(xd))
    e_op = maxrel(y, ax)
    assert e_op <= tol
    r = host(P.residual(to_dev(poisoned(b, d, k, L), dtype), xd))
    e_res = maxrel(r, b - ax)
    assert e_res <= tol
    bm = mesh.boundary_mask(d, k, L)
    assert np.all(y[bm] == 0.0) and np.all(r[bm] == 0.0)
    print("  max error / max |ref|: apply %.2e residual %.2e" % (e_op, e_res), flush=True)


# ------------------------------------------------------------------ transfers, several tiles per axis

# 3D restriction tiles hold K * CX coarse columns (16, 16, 15, 16, 15, 12, 14 for K = 1..7): these
# levels give 2..8 tiles per axis, ragged (3D Q3, Q5) and exact multiples (the others).  In FP32 the
# plane pass takes two fine planes per workgroup, and the number of interior fine planes is odd, so
# its last group is partial at every level.
# 2D prolongation tiles hold (32, 16, 8, 8, 4, 4, 4) coarse cells per axis for K = 1..7: the 2D
# levels below give 2..8 tiles per axis.
TRANSFER_CASES = [(3, 1, 6), (3, 2, 5), (3, 3, 5), (3, 4, 4), (3, 4, 6), (3, 5, 4), (3, 6, 4), (3, 7, 4),
                  (3, 7, 5), (2, 3, 7), (2, 7, 6), (2, 1, 7), (2, 2, 6), (2, 4, 6), (2, 5, 5), (2, 6, 5)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,L", TRANSFER_CASES)
def test_transfer_several_tiles(d, k, L, prec):
    dtype = F64 if prec == "fp64" else F32
    tol = 1e-12 if prec == "fp64" else 2e-6
    case("transfer", d, k, L, prec)
    P = problem(d, k, L)
    r = as_seen(synth.random_interior(d, k, L, 121), dtype)
    e = as_seen(synth.random_interior(d, k, L - 1, 122), dtype)
    x = as_seen(synth.random_interior(d, k, L, 123), dtype)
    rc = host(P.restrict(to_dev(poisoned(r, d, k, L), dtype)))
    e_res = maxrel(rc, transfer.restrict(d, k, L, r))
    assert e_res <= tol
    assert np.all(rc[mesh.boundary_mask(d, k, L - 1)] == 0.0)
    xt = to_dev(x, dtype)
    P.prolongate_add(to_dev(poisoned(e, d, k, L - 1), dtype), xt)
    ref = x + transfer.prolongate(d, k, L, e)
    e_pro = maxrel(host(xt), ref)
    assert e_pro <= tol
    print("  max error / max |ref|: restrict %.2e prolongate %.2e" % (e_res, e_pro), flush=True)


# ------------------------------------------------------------------ matrix-core form of the colour pass

@pytest.mark.parametrize("d,k,L", [(3, 4, 6), (3, 4, 5)])
def test_mfma_colour_pass_every_patch(d, k, L):
    """VPS_MULTIPLICATIVE_MFMA (residual contractions on the matrix cores, 3D Q4 FP32, launches of
    at least 1024 workgroups; smaller colours take the vector form) against the oracle, every patch
    of every colour, same bar as the vector form."""
    dtype, tol = F32, TOL32[d]
    P = problem(d, k, L)
    b = as_seen(synth.random_interior(d, k, L, 131), dtype)
    x = as_seen(synth.random_interior(d, k, L, 132), dtype)
    bd = to_dev(poisoned(b, d, k, L), dtype)
    x_pois = poisoned(x, d, k, L)
    worst = 0.0
    for c in range(2 ** d):
        case("mfma colour pass", d, k, L, "colour", c)
        verts = mesh.patches_of_colour(d, L, c)
        C = mesh.patch_box_ids_many(d, k, L, verts, interior=False)
        I = mesh.patch_box_ids_many(d, k, L, verts, interior=True)
        ref = smoother.patch_update_local_many(d, k, L, x[C], b[I])
        outside = np.ones(x.shape, dtype=bool)
        outside[I.reshape(-1)] = False
        xt = to_dev(x_pois, dtype)
        P.color_pass(bd, xt, c, vps.VPS_MULTIPLICATIVE_MFMA)
        got = host(xt)
        e = maxrel(got[I], ref)
        worst = max(worst, e)
        assert e <= tol, (c, e)
        assert np.array_equal(got[outside], x_pois[outside], equal_nan=True), c
    print("  max error / max |ref|: %.2e" % worst, flush=True)


@pytest.mark.parametrize("d,k,L,dtype", [(3, 3, 5, F32), (3, 4, 6, F64), (2, 4, 6, F32)])
def test_mfma_mode_elsewhere_is_the_vector_pass(d, k, L, dtype):
    """Where the matrix-core form does not exist, VPS_MULTIPLICATIVE_MFMA runs the vector pass: bit
    for bit the same as VPS_MULTIPLICATIVE."""
    case("mfma fallback", d, k, L, dtype)
    P = problem(d, k, L)
    b = to_dev(synth.random_interior(d, k, L, 141), dtype)
    x0 = to_dev(synth.random_interior(d, k, L, 142), dtype)
    for c in range(2 ** d):
        x1, x2 = x0.clone(), x0.clone()
        P.color_pass(b, x1, c, vps.VPS_MULTIPLICATIVE)
        P.color_pass(b, x2, c, vps.VPS_MULTIPLICATIVE_MFMA)
        torch.cuda.synchronize()
        assert torch.equal(x1, x2), c
