"""GPU "Separate" smoother (Sec. 4.1, Table 6): per colour the residual kernel, then the local solves.

Bars: FP64 within 1e-12 (2-norm, relative) of the oracle's multiplicative colour pass, smoother and
V-cycle; FP32 within 1e-5; CG with the Separate V-cycle converges like the fused one.
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

F64, F32 = torch.float64, torch.float32
SEP = vps.VPS_MULTIPLICATIVE_SEPARATE


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


@pytest.mark.parametrize("d,k,L", [(2, 1, 4), (2, 3, 3), (2, 7, 2), (3, 1, 3), (3, 2, 3), (3, 4, 2), (3, 6, 2),
                                   (3, 4, 1)])
def test_separate_colour_pass(d, k, L):
    case("separate colour pass", d, k, L)
    P = vps.Problem(d, k, L, vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY | vps.VPS_FLAG_NO_SOLVER)
    b = synth.random_interior(d, k, L, 51)
    x = synth.random_interior(d, k, L, 52)
    for c in range(2 ** d):
        ref = smoother.colour_pass(d, k, L, b, x, c)
        xt = dev(x)
        P.color_pass(dev(b), xt, c, SEP, level=L)
        assert rel(host(xt), ref) <= 1e-12, c
        xt = dev(x, F32)
        P.color_pass(dev(b, F32), xt, c, SEP, level=L)
        assert rel(host(xt), ref) <= 1e-5, c
    P.close()


@pytest.mark.parametrize("d,k,L", [(2, 2, 4), (3, 2, 3), (3, 4, 2)])
def test_separate_smoother_vcycle_and_cg(d, k, L):
    case("separate smoother in V-cycle", d, k, L)
    flags = vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY
    P = vps.Problem(d, k, L, flags | vps.VPS_FLAG_SEPARATE_SMOOTHER)
    b = synth.random_interior(d, k, L, 53)
    x = synth.random_interior(d, k, L, 54)
    for rev in (False, True):
        xt = dev(x)
        P.smoother_apply(dev(b), xt, SEP, rev)
        assert rel(host(xt), smoother.multiplicative(d, k, L, b, x, reverse=rev)) <= 1e-12
    ref = multigrid.vcycle(d, k, L, b, x)
    xt = dev(x)
    P.vcycle(dev(b), xt)
    assert rel(host(xt), ref) <= 1e-12
    xt = dev(x, F32)
    P.vcycle(dev(b, F32), xt)
    assert rel(host(xt), ref) <= 1e-5
    Pf = vps.Problem(d, k, L, flags)
    for mode in (vps.VPS_SOLVE_FP64, vps.VPS_SOLVE_MIXED):
        x1, s1 = P.pcg_solve(dev(b), rtol=1e-10, mode=mode)
        x2, s2 = Pf.pcg_solve(dev(b), rtol=1e-10, mode=mode)
        assert s1.status == 0 and abs(s1.iterations - s2.iterations) <= 1
        assert rel(host(x1), host(x2)) <= 1e-8
    Pf.close()
    P.close()


def test_separate_needs_the_hierarchy_of_its_precision():
    P = vps.Problem(2, 2, 3, vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_NO_SOLVER)
    b = torch.zeros(P.n(), dtype=F32, device="cuda")
    with pytest.raises(vps.VpsError):
        P.color_pass(b, b.clone(), 0, SEP)
    P.close()
