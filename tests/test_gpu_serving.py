"""Serving (continuous batching) on the GPU: results alone == in the mix, admission by memory budget."""
import numpy as np
import pytest

import synth
from oracle import mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_19004_amd as vps  # noqa: E402

SHAPES = [(2, 1, 7), (3, 2, 3), (2, 7, 4), (3, 4, 3), (2, 3, 6), (3, 1, 5), (3, 6, 2), (2, 5, 5),
          (3, 2, 4), (2, 3, 4), (3, 4, 2)]


def _rhs(d, k, L, seed):
    P = vps.Problem(d, k, L, vps.VPS_FLAG_FP32_HIERARCHY | vps.VPS_FLAG_NO_SOLVER)
    kap, co = synth.fourier_modes(d, seed=seed)
    b = P.rhs_sine_modes(kap, co)
    P.close()
    return b


def _alone(d, k, L, b, mode):
    P = vps.Problem(d, k, L)
    x, st = P.pcg_solve(b, rtol=1e-8, mode=mode)
    torch.cuda.synchronize()
    out = x.clone(), st.iterations, st.status
    P.close()
    return out


def _serve(reqs, budget, max_active, mode):
    srv = vps.vps_server_create(budget, max_active)
    xs, tickets = [], []
    peak = 0
    try:
        for (d, k, L), b in reqs:
            x = torch.full_like(b, 5.0)
            xs.append(x)
            tickets.append(vps.vps_server_submit(srv, d, k, L, b.data_ptr(), x.data_ptr(), 1e-8, mode, 50))
        finished = []
        for _ in range(10000):
            active, queued = vps.vps_server_step(srv)
            in_use, cached = vps.vps_server_memory(srv)
            peak = max(peak, in_use + cached)
            finished += vps.vps_server_completed(srv, cap=3)  # small cap: several calls per tick
            if active == 0 and queued == 0:
                break
        stats = [vps.vps_server_poll(srv, t) for t in tickets]
        # every ticket is reported exactly once, and only once it is done
        assert sorted(finished) == sorted(tickets) and vps.vps_server_completed(srv) == []
    finally:
        vps.vps_server_destroy(srv)
    return xs, stats, peak


@pytest.mark.parametrize("mode", [vps.VPS_SOLVE_MIXED, vps.VPS_SOLVE_FP64])
def test_results_identical_alone_and_in_the_mix(mode):
    reqs = [((d, k, L), _rhs(d, k, L, 100 + i)) for i, (d, k, L) in enumerate(SHAPES)]
    reqs += reqs[:3]  # repeated shapes reuse cached hierarchies
    xs, stats, _ = _serve(reqs, 8 << 30, 6, mode)
    for ((d, k, L), b), x, (done, st) in zip(reqs, xs, stats):
        print("request", d, k, L, st.iterations, st.status, flush=True)
        assert done and st.status == 0
        ref, its, status = _alone(d, k, L, b, mode)
        assert status == 0 and its == st.iterations
        assert torch.equal(x, ref)  # deterministic kernels: bitwise identical
        bh = b.cpu().numpy()
        r = bh - mesh.apply_operator(d, k, L, x.cpu().numpy())
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(bh)


def test_admission_respects_a_tight_budget():
    reqs = [((3, 2, 4), _rhs(3, 2, 4, 7)), ((3, 3, 4), _rhs(3, 3, 4, 8)), ((2, 4, 6), _rhs(2, 4, 6, 9))]
    need = max(vps.vps_footprint_bytes(d, k, L, vps.VPS_FLAG_FP32_HIERARCHY) for (d, k, L), _ in reqs)
    budget = int(need * 1.2)  # room for one request at a time
    xs, stats, peak = _serve(reqs, budget, 8, vps.VPS_SOLVE_MIXED)
    assert peak <= budget
    for (done, st) in stats:
        assert done and st.status == 0


def test_bad_requests_fail_alone():
    b_ok = _rhs(2, 2, 4, 11)
    b_nan = b_ok.clone()
    b_nan[300] = float("nan")
    srv = vps.vps_server_create(1 << 30, 4)
    try:
        with pytest.raises(vps.VpsError) as e:
            vps.vps_server_submit(srv, 3, 7, 8, b_ok.data_ptr(), b_ok.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        assert e.value.status == vps.VPS_EBUSY
        x1, x2 = torch.zeros_like(b_ok), torch.zeros_like(b_ok)
        t1 = vps.vps_server_submit(srv, 2, 2, 4, b_nan.data_ptr(), x1.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        t2 = vps.vps_server_submit(srv, 2, 2, 4, b_ok.data_ptr(), x2.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        for _ in range(100):
            a, q = vps.vps_server_step(srv)
            if a == 0 and q == 0:
                break
        d1, s1 = vps.vps_server_poll(srv, t1)
        d2, s2 = vps.vps_server_poll(srv, t2)
        assert d1 and s1.status == vps.VPS_ENOTFINITE
        assert d2 and s2.status == 0
    finally:
        vps.vps_server_destroy(srv)


def test_zero_rhs_request_finishes_at_admission():
    # b = 0: the solve ends at its set-up (x = 0, no iteration); a request beside it is unaffected
    b_ok = _rhs(3, 2, 3, 12)
    b_zero = torch.zeros_like(b_ok)
    x_ref, its_ref, st_ref = _alone(3, 2, 3, b_ok, vps.VPS_SOLVE_MIXED)
    srv = vps.vps_server_create(1 << 30, 4)
    try:
        x0, x1 = torch.full_like(b_ok, 5.0), torch.full_like(b_ok, 5.0)
        t0 = vps.vps_server_submit(srv, 3, 2, 3, b_zero.data_ptr(), x0.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        t1 = vps.vps_server_submit(srv, 3, 2, 3, b_ok.data_ptr(), x1.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        vps.vps_server_step(srv)
        d0, s0 = vps.vps_server_poll(srv, t0)
        assert d0 and s0.status == 0 and s0.iterations == 0 and s0.rel_residual == 0.0
        for _ in range(200):
            a, q = vps.vps_server_step(srv)
            if a == 0 and q == 0:
                break
        d1, s1 = vps.vps_server_poll(srv, t1)
        torch.cuda.synchronize()
        assert torch.count_nonzero(x0).item() == 0
        assert d1 and s1.status == st_ref and s1.iterations == its_ref
        assert torch.equal(x1, x_ref)
    finally:
        vps.vps_server_destroy(srv)


def test_rhs_written_on_the_caller_stream_just_before_submit():
    """The server orders a request's first read of b after the work queued on the caller's stream
    at submit: b is filled by a copy queued behind a ~20 ms spin on that stream, and the request
    still solves the filled rhs (an unordered read would see zeros and end at once with x = 0)."""
    d, k, L = 2, 3, 5
    src = _rhs(d, k, L, 21)
    x_ref, its_ref, st_ref = _alone(d, k, L, src, vps.VPS_SOLVE_MIXED)
    s = torch.cuda.Stream()
    srv = vps.vps_server_create(1 << 30, 4, s.cuda_stream)
    try:
        b = torch.zeros_like(src)
        x = torch.zeros_like(src)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            torch.cuda._sleep(40_000_000)
            b.copy_(src)
            t = vps.vps_server_submit(srv, d, k, L, b.data_ptr(), x.data_ptr(), 1e-8, vps.VPS_SOLVE_MIXED, 50)
        for _ in range(200):
            a, q = vps.vps_server_step(srv)
            if a == 0 and q == 0:
                break
        done, st = vps.vps_server_poll(srv, t)
        assert done and st.status == st_ref and st.iterations == its_ref > 0
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref)
    finally:
        vps.vps_server_destroy(srv)


def test_failed_requests_leave_the_server_consistent():
    """Launch failures forced from the host (vps_server_inject_fault) at admission, at a CG
    iteration and in a preconditioner: each failing request ends with the error as its status and
    gives its hierarchy back; the requests beside it finish bitwise as they do alone; no memory
    stays counted as in use; and the server serves the same shapes again afterwards."""
    shapes = [(2, 3, 5), (3, 2, 3), (2, 5, 4), (3, 4, 2), (2, 3, 5)]
    stage = {0: 0, 1: 1, 2: 2}  # request index -> the stage whose launch fails
    bs = [_rhs(d, k, L, 30 + i) for i, (d, k, L) in enumerate(shapes)]
    mode = vps.VPS_SOLVE_MIXED
    srv = vps.vps_server_create(4 << 30, 8)
    try:
        xs = [torch.full_like(b, 5.0) for b in bs]
        ts = [vps.vps_server_submit(srv, d, k, L, b.data_ptr(), x.data_ptr(), 1e-8, mode, 50)
              for (d, k, L), b, x in zip(shapes, bs, xs)]
        for i, sg in stage.items():
            vps.vps_server_inject_fault(srv, ts[i], sg)
        for _ in range(500):
            a, q = vps.vps_server_step(srv)
            if a == 0 and q == 0:
                break
        res = [vps.vps_server_poll(srv, t) for t in ts]
        for i, (done, st) in enumerate(res):
            print("request", i, shapes[i], "status", st.status, "iterations", st.iterations, flush=True)
            assert done
            if i in stage:
                assert st.status == vps.VPS_EHIP
            else:
                ref, its, status = _alone(*shapes[i], bs[i], mode)
                assert st.status == status == 0 and st.iterations == its
                assert torch.equal(xs[i], ref)
        in_use, cached = vps.vps_server_memory(srv)
        assert in_use == 0 and cached > 0
        with pytest.raises(vps.VpsError):
            vps.vps_server_inject_fault(srv, ts[0], 1)  # finished
        # the shapes of the failed requests are served again, from the cached hierarchies
        again = [0, 2]
        xs2 = [torch.zeros_like(bs[i]) for i in again]
        ts2 = [vps.vps_server_submit(srv, *shapes[i], bs[i].data_ptr(), x.data_ptr(), 1e-8, mode, 50)
               for i, x in zip(again, xs2)]
        for _ in range(500):
            a, q = vps.vps_server_step(srv)
            if a == 0 and q == 0:
                break
        for i, x, t in zip(again, xs2, ts2):
            done, st = vps.vps_server_poll(srv, t)
            ref, its, status = _alone(*shapes[i], bs[i], mode)
            assert done and st.status == 0 and st.iterations == its
            assert torch.equal(x, ref)
        assert vps.vps_server_memory(srv)[0] == 0
    finally:
        vps.vps_server_destroy(srv)
