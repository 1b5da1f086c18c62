"""GPU "Boundary" colour pass (Sec. 4.1.3, eq:A_ib_2d/3d) against the FP64 oracle.

The kernel overwrites each patch interior with A_j^{-1}(b^I - A^{IB} x^B).  Bars: FP64 within
1e-12 (2-norm, relative) of the oracle's Boundary pass (itself pinned to the fused pass and to
the assembled A^{IB}); FP32 within 1e-5.  The old interior values are never read: NaN planted
in them leaves the result bitwise unchanged.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import multigrid, smoother

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402
from oracle import mesh  # noqa: E402

F64, F32 = torch.float64, torch.float32
BND = vps.VPS_MULTIPLICATIVE_BOUNDARY


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


CASES = [(2, 1, 5), (2, 2, 4), (2, 3, 3), (2, 4, 3), (2, 5, 2), (2, 6, 2), (2, 7, 2),
         (3, 1, 3), (3, 2, 3), (3, 3, 2), (3, 4, 2), (3, 5, 2), (3, 6, 2), (3, 7, 2)]


@pytest.mark.parametrize("d,k,L", CASES)
def test_boundary_colour_pass(d, k, L):
    case("boundary colour pass", d, k, L)
    P = vps.Problem(d, k, L, vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY | vps.VPS_FLAG_NO_SOLVER)
    b = synth.random_interior(d, k, L, 41)
    x = synth.random_interior(d, k, L, 42)
    for c in range(2 ** d):
        ref = smoother.colour_pass_boundary(d, k, L, b, x, c)
        xt = dev(x)
        P.color_pass(dev(b), xt, c, BND)
        assert rel(host(xt), ref) <= 1e-12, c
        xt = dev(x, F32)
        P.color_pass(dev(b, F32), xt, c, BND)
        assert rel(host(xt), ref) <= 1e-5, c
    P.close()


@pytest.mark.parametrize("d,k,L", [(2, 3, 4), (3, 2, 3), (3, 4, 2), (3, 7, 2)])
def test_boundary_pass_never_reads_the_interior(d, k, L):
    case("boundary pass with NaN interiors", d, k, L)
    P = vps.Problem(d, k, L, vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_NO_SOLVER)
    b = dev(synth.random_interior(d, k, L, 43))
    x = synth.random_interior(d, k, L, 44)
    for c in range(2 ** d):
        verts = mesh.patches_of_colour(d, L, c)
        if len(verts) == 0:
            continue
        I = np.concatenate([mesh.patch_interior_ids(d, k, L, v) for v in verts])
        xn = x.copy()
        xn[I] = np.nan
        clean, poisoned = dev(x), dev(xn)
        P.color_pass(b, clean, c, BND)
        P.color_pass(b, poisoned, c, BND)
        assert torch.equal(clean, poisoned), c
    P.close()


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (2, 5, 3), (3, 2, 3), (3, 3, 3), (3, 4, 2)])
def test_boundary_smoother_in_vcycle_and_solvers(d, k, L):
    case("boundary smoother in V-cycle", d, k, L)
    flags = vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY | vps.VPS_FLAG_BOUNDARY_SMOOTHER
    P = vps.Problem(d, k, L, flags)
    b = synth.random_interior(d, k, L, 45)
    x = synth.random_interior(d, k, L, 46)
    # one smoothing step, both colour orders
    for rev in (False, True):
        xt = dev(x)
        P.smoother_apply(dev(b), xt, BND, rev)
        assert rel(host(xt), smoother.multiplicative(d, k, L, b, x, reverse=rev)) <= 1e-12
    # V-cycle (symmetric order) in FP64 and FP32
    ref = multigrid.vcycle(d, k, L, b, x)
    xt = dev(x)
    P.vcycle(dev(b), xt)
    assert rel(host(xt), ref) <= 1e-12
    xt = dev(x, F32)
    P.vcycle(dev(b, F32), xt)
    assert rel(host(xt), ref) <= 1e-5
    # CG with the V-cycle: same iterates as the fused smoother within rounding
    Pf = vps.Problem(d, k, L, flags & ~vps.VPS_FLAG_BOUNDARY_SMOOTHER)
    for mode in (vps.VPS_SOLVE_FP64, vps.VPS_SOLVE_MIXED):
        x1, s1 = P.pcg_solve(dev(b), rtol=1e-10, mode=mode)
        x2, s2 = Pf.pcg_solve(dev(b), rtol=1e-10, mode=mode)
        assert s1.status == 0 and abs(s1.iterations - s2.iterations) <= 1
        assert rel(host(x1), host(x2)) <= 1e-8
    Pf.close()
    P.close()
