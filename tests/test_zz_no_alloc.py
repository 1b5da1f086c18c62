"""The allocation-free restriction (vps_restrict_noalloc) through the C-ABI: its output equals the
problem-owned restriction (vps_restrict) bit for bit on the same input, for two calls in a row
(the second smaller, so the shared scratch holds the first call's larger intermediate), in both
precisions and dimensions; sizes beyond its scratch are refused on the host."""
import sys

import numpy as np
import pytest

import synth
from oracle import mesh, transfer

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402

PREC = {torch.float64: vps.VPS_FP64, torch.float32: vps.VPS_FP32}


def _pair(d, k, L, dtype, seed):
    print("case no-alloc restrict", d, k, L, dtype, flush=True)
    sys.stdout.flush()
    r = synth.random_interior(d, k, L, seed)
    rf = torch.from_numpy(r).to(device="cuda", dtype=dtype)
    P = vps.Problem(d, k, L)
    ref = P.restrict(rf)  # the problem-owned entry point
    out = torch.full((mesh.n1d(k, L - 1) ** d,), float("nan"), dtype=dtype, device="cuda")
    s = torch.cuda.current_stream()
    vps.vps_restrict_noalloc(d, k, L, PREC[dtype], rf.data_ptr(), out.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    P.close()
    return r, ref, out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_restrict_equals_the_problem_entry_point_twice(dtype):
    # first the largest intermediate of the cases (3D Q4, 64^3 cells), then smaller ones
    for d, k, L, seed in [(3, 4, 6, 71), (3, 2, 4, 72), (2, 7, 5, 73)]:
        r, ref, out = _pair(d, k, L, dtype, seed)
        assert torch.equal(out, ref), (d, k, L)
        tol = 1e-12 if dtype == torch.float64 else 2e-6
        if L <= 4 or d == 2:  # oracle check on the small cases
            exp = transfer.restrict(d, k, L, r.astype(np.float32).astype(np.float64) if dtype == torch.float32 else r)
            got = out.double().cpu().numpy()
            assert np.max(np.abs(got - exp)) <= tol * np.max(np.abs(exp))


def test_noalloc_restrict_refuses_sizes_beyond_its_scratch():
    with pytest.raises(vps.VpsError) as e:
        vps.vps_restrict_noalloc(3, 4, 7, vps.VPS_FP64, 1, 1, None)  # 513 x 257^2 doubles > 64 MiB
    assert e.value.status == vps.VPS_EINVAL and "exceeds" in str(e.value)
