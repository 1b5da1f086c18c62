"""The CG preconditioner replayed from a captured HIP graph gives exactly the eagerly launched result.

Every solve replays the graph once per CG iteration with the CG's own kernels and a host
synchronisation in between; each of several consecutive solves (and both solve modes) with
VPS_FLAG_GRAPHS must be bitwise identical to the same solve with direct launches.
"""
import sys

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402


@pytest.mark.parametrize("d,k,L", [(3, 4, 4), (2, 3, 5), (3, 2, 3)])
@pytest.mark.parametrize("order", [0, vps.VPS_FLAG_POST_SAME_ORDER])
def test_graph_replays_match_eager_solves(d, k, L, order):
    print("case graphs", d, k, L, order, flush=True)
    sys.stdout.flush()
    base = vps.VPS_FLAG_FP64_HIERARCHY | vps.VPS_FLAG_FP32_HIERARCHY | order
    Pg = vps.Problem(d, k, L, base | vps.VPS_FLAG_GRAPHS)
    Pe = vps.Problem(d, k, L, base)
    kap, co = synth.fourier_modes(d, seed=3)
    b = Pg.rhs_sine_modes(kap, co)
    for mode in (vps.VPS_SOLVE_MIXED, vps.VPS_SOLVE_FP64):
        xe, se = Pe.pcg_solve(b, rtol=1e-10, mode=mode)
        torch.cuda.synchronize()
        for rep in range(3):
            xg, sg = Pg.pcg_solve(b, rtol=1e-10, mode=mode)
            torch.cuda.synchronize()
            assert sg.status == 0 and sg.iterations == se.iterations, (rep, sg.iterations, se.iterations)
            assert torch.equal(xg, xe), rep
            # eager work on the same stream between replays
            b2 = b * 0.5
            Pg.operator_apply(b2, torch.empty_like(b2))
            torch.cuda.synchronize()
    Pg.close()
    Pe.close()
