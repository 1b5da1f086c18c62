"""Benchmark: vertex-patch multigrid on one MI355X.

Workload: 3D Poisson, Q4 elements on 64^3 cells of the unit cube (257^3 =
16,974,593 nodes), right-hand side a seeded sum of 16 Fourier sine modes with
amplitudes decaying as |kappa|^-2 (seed 1).

A step is one full mixed-precision solve: CG in FP64 preconditioned by one FP32
V-cycle (multiplicative vertex-patch smoother, matrix-free operator, transfers,
FP64 coarse solve) until ||r|| <= 1e-8 ||b||, from b resident in HBM to x in
HBM.  The V-cycle applies the same colour order before and after the coarse
correction (Alg. 1 read literally) and CG uses the flexible beta.  value =
nodes x steps / timed seconds.  The symmetric V-cycle (reversed colours after the
correction) and the FP64 solves are measured beside it.  Outside the timed region the
script also measures the FP64 solve, one smoothing step and one V-cycle in each
precision, the colour-pass kernel for the roofline, a short serving run
(continuous batching, p50/p99 latency) and the CPU oracle on a bounded sample.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D, K, L = 3, 4, 6
RTOL = 1e-8
PEAK_FP32 = 157.3e12  # MI355X published FP32 vector peak
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12  # MI355X HBM3E
# LDS: bytes per clock and compute unit as assumed for CDNA3-class LDS (32 banks of 4 bytes); the
# record states the figure next to the fraction
LDS_BYTES_PER_CLK = 128
PEAK_LDS = LDS_BYTES_PER_CLK * 256 * 2.4e9


def smoother_patch_flops(d, k):
    """Algorithmic flops of one patch update (the measurement model of the smoother): the residual
    on the patch-interior rows by sum factorisation with the partial products reused across
    directions (Sec. 3.1.1), the fast-diagonalisation solve (S^T and S along every direction,
    eq:inverse2d/3d, plus the eigenvalue scaling) and the update, every 1D matrix taken dense:
      2D: 2 (2 n^2 m + 2 n m^2 + 4 m^3) + 2 m^2,
      3D: 2 (2 n^3 m + 3 n^2 m^2 + 2 n m^3 + 6 m^4) + 2 m^3,   n = 2k+1, m = 2k-1."""
    n, m = 2 * k + 1, 2 * k - 1
    if d == 3:
        return 2 * (2 * n ** 3 * m + 3 * n * n * m * m + 2 * n * m ** 3 + 6 * m ** 4) + 2 * m ** 3
    return 2 * (2 * n * n * m + 2 * n * m * m + 4 * m ** 3) + 2 * m * m


def smoother_patch_min_words(d, k):
    """Minimum HBM words of one patch update: x on the closure skeleton and b on the interior read,
    x on the interior written, (2k+1)^d + (2k-1)^d (each colour touches each node about once)."""
    return (2 * k + 1) ** d + (2 * k - 1) ** d


def colour_pass_issued_flops(d, k):
    """Flops the colour-pass kernel executes per patch (smoother_patch_flops without the products
    with structural zeros and with the eigenvector symmetry used).  The 1D patch rows have
    nnz = (2k-2)(k+1) + (2k+1) structural nonzeros (a cell-interior node couples to its cell's
    k+1 nodes, the middle vertex to all 2k+1); products with structural zeros are not counted.
    The eigenvectors are even or odd under the patch mirror, so one application of S or S^T to a
    line takes (m^2+1)/2 multiply-adds and m-1 additions.  fma = 2 flops, mul/add = 1."""
    n, m = 2 * k + 1, 2 * k - 1
    nnz = (2 * k - 2) * (k + 1) + (2 * k + 1)
    s_fma, s_add = (m * m + 1) // 2, m - 1
    if d == 3:
        fma = 2 * nnz * n * n + 3 * nnz * n * m + 2 * nnz * m * m + m ** 3 + 6 * m * m * s_fma + m ** 3
        mul, add = m ** 3, 6 * m * m * s_add
    else:
        fma = 2 * nnz * n + 2 * nnz * m + m * m + 4 * m * s_fma + m * m
        mul, add = m * m, 4 * m * s_add
    return 2 * fma + mul + add


def colour_pass_bytes(d, k, es):
    """Algorithmic HBM bytes of one patch: read x closure + b interior, write x interior."""
    n, m = 2 * k + 1, 2 * k - 1
    return es * (n ** d + 2 * m ** d)


def colour_pass_lds_bytes_3d(k, es, ppw):
    """LDS bytes one patch moves in the 3D colour pass that runs the closure through LDS (every
    write and read of its stages): closure rows in, then per stage the lines read and written."""
    n, m = 2 * k + 1, 2 * k - 1
    words = n * n * (2 * k * ppw + 1) / ppw    # closure segment written (shared faces once)
    words += n ** 3 + 2 * n * n * m            # x0: closure lines in, M and A rows out
    words += 2 * n * n * m + 2 * n * m * m     # x1
    words += 2 * n * m * m + m ** 3            # x2 residual and S^T along x2
    words += 2 * m ** 3 * 3                    # S^T x1; S^T x0, 1/lambda, S x0; S x1
    words += 2 * m ** 3                        # S x2, and the old interior values from the closure
    return es * words


def smoother_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("smoother.hip", "device_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2405_19004_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--serve", type=int, default=2000, help="requests in the serving run (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-table7", action="store_true",
                    help="skip the mixed/double solves at the sizes of Table 7 (135M-721M DoFs)")
    ap.add_argument("--quick", action="store_true", help="only the timed solves (for profiling)")
    ap.add_argument("--quick-2d", action="store_true",
                    help="only the 2D Q7 512^2 solves, mixed and FP64 (for profiling)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the closed-loop mixed serving run of --serve requests (for profiling)")
    ap.add_argument("--serve-slots", type=int, default=16, help="requests the server keeps active at once")
    ap.add_argument("--serve-replays", action="store_true",
                    help="with --serve-only: every replay (Poisson, FP64, one at a time), not only the closed loop")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only 8 FP32 and 8 FP64 colour passes on the finest level, twice (for counter runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only a plain device copy of this many MiB, 4 times (counter calibration)")
    return ap.parse_args()


def event_time(fn, stream, reps):
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps / 1e3


def progress(msg):
    """One line per finished phase on stderr (the JSON result alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def serving_run(v, n_requests, max_active=16, budget=64 << 30, closed_loop_only=False):
    """Continuous-batching server over a seeded stream of mixed (d, k, level) requests.

    Right-hand sides are assembled on the device before the clock starts.  First a closed-loop
    run (every request present at t = 0) measures capacity; then the same requests arrive as a
    Poisson process at 80 % of that capacity and latency (arrival -> completion) is recorded per
    request.  The same arrival trace is replayed with plain FP64 solves, and one request at a time
    (no batching, one slot); a closed-loop FP64 run gives the FP64 capacity.  Every request's
    status and true residual are checked: a request that did not converge is counted as failed.
    """
    import synth
    trace = synth.serving_trace(seed=3, n_requests=n_requests, rate_per_s=1.0)
    makers = {}
    for r in trace:
        key = (r["d"], r["k"], r["level"])
        if key not in makers:
            makers[key] = v.Problem(r["d"], r["k"], r["level"], v.VPS_FLAG_FP32_HIERARCHY | v.VPS_FLAG_NO_SOLVER)
        P = makers[key]
        r["b"] = P.rhs_sine_modes(r["kappas"], r["coefs"])
        r["x"] = P.new()
        r["n"] = P.n()
    for P in makers.values():
        P.close()
    import torch
    torch.cuda.synchronize()
    sizes = [r["n"] for r in trace]
    classes = [(1e4, 1e5), (1e5, 1e6), (1e6, 1e7 + 1)]

    def run(scale, mode=v.VPS_SOLVE_MIXED, slots=max_active):
        srv = v.vps_server_create(budget, slots)
        t0 = time.perf_counter()
        pending = list(range(len(trace)))
        arrive, done, ticket_of = {}, {}, {}
        try:
            while True:
                now = time.perf_counter() - t0
                while pending and trace[pending[0]]["arrival"] * scale <= now:
                    i = pending.pop(0)
                    r = trace[i]
                    t = v.vps_server_submit(srv, r["d"], r["k"], r["level"], r["b"].data_ptr(), r["x"].data_ptr(),
                                            RTOL, mode, 50)
                    arrive[t] = r["arrival"] * scale
                    ticket_of[t] = i
                active, queued = v.vps_server_step(srv)
                now = time.perf_counter() - t0
                for t in v.vps_server_completed(srv):
                    done[t] = now
                if not pending and len(done) == len(trace):
                    break
                if active == 0 and queued == 0 and pending:
                    time.sleep(max(0.0, trace[pending[0]]["arrival"] * scale - (time.perf_counter() - t0)))
            span = time.perf_counter() - t0
            failed, worst = 0, 0.0
            for t in done:
                _, st = v.vps_server_poll(srv, t)
                if st.status != 0 or not st.true_rel_residual <= 1.01 * RTOL:
                    failed += 1
                worst = max(worst, st.true_rel_residual)
        finally:
            v.vps_server_destroy(srv)
        lat = {ticket_of[t]: done[t] - arrive[t] for t in done}
        return span, lat, failed, worst

    def q(a, p):
        a = sorted(a)
        return a[min(len(a) - 1, int(round(p * (len(a) - 1))))] if a else None

    def summary(span, lat, failed, worst):
        vals = list(lat.values())
        out = {"makespan_s": span, "dof_per_s": sum(sizes) / span, "req_per_s": len(trace) / span,
               "p50_ms": 1e3 * q(vals, 0.5), "p99_ms": 1e3 * q(vals, 0.99), "mean_ms": 1e3 * sum(vals) / len(vals),
               "failed": failed, "worst_true_rel_residual": worst, "by_size": {}}
        for lo, hi in classes:
            sel = [lat[i] for i in lat if lo <= sizes[i] < hi]
            if sel:
                out["by_size"]["%.0e-%.0e" % (lo, min(hi, 1e7))] = {
                    "requests": len(sel), "p50_ms": 1e3 * q(sel, 0.5), "p99_ms": 1e3 * q(sel, 0.99)}
        return out

    total = sum(sizes)
    closed = run(0.0)
    if closed_loop_only:
        return {"requests": len(trace), "total_dofs": total, "max_active": max_active,
                "closed_loop_mixed": summary(*closed)}
    capacity = len(trace) / closed[0]
    rate = 0.8 * capacity
    res = {"requests": len(trace), "total_dofs": total, "max_active": max_active, "arrival_rate_per_s": rate}
    res["closed_loop_mixed"] = summary(*closed)
    res["poisson_mixed"] = summary(*run(1.0 / rate))
    res["poisson_fp64"] = summary(*run(1.0 / rate, v.VPS_SOLVE_FP64))
    res["poisson_mixed_one_at_a_time"] = summary(*run(1.0 / rate, v.VPS_SOLVE_MIXED, 1))
    res["closed_loop_fp64"] = summary(*run(0.0, v.VPS_SOLVE_FP64))
    res["mixed_vs_fp64_closed_loop_speedup"] = res["closed_loop_fp64"]["makespan_s"] / closed[0]
    # headline figures of the Poisson replay at 80 % of the mixed capacity
    res["p50_ms"], res["p99_ms"] = res["poisson_mixed"]["p50_ms"], res["poisson_mixed"]["p99_ms"]
    res["dof_per_s"] = res["poisson_mixed"]["dof_per_s"]
    res["failed"] = sum(res[k]["failed"] for k in res if isinstance(res[k], dict) and "failed" in res[k])
    return res


# Table 7 (3D, manufactured solution prod sin(pi x_i), residual reduction 1e-9): degree,
# level, and the printed double / mixed L2 error, iterations and seconds (other hardware).
TABLE7 = [(1, 9, 1.12e-06, 5, 3.391, 5, 2.385), (3, 8, 2.30e-13, 3, 3.941, 3, 2.418),
          (7, 7, 2.89e-16, 2, 5.891, 2, 3.326)]


def table7_run(v, torch):
    """Solves of Table 7's three problems in both precisions: time (rhs resident, solve only),
    CG iterations and L2 error of the discrete solution."""
    import synth
    rows = []
    for k, lev, l2_paper, it64_p, t64_p, itmx_p, tmx_p in TABLE7:
        kap, co = synth.manufactured_sine(3)
        uc = [c / (math.pi ** 2 * sum(q * q for q in kk)) for kk, c in zip(kap, co)]
        P = v.Problem(3, k, lev, v.VPS_FLAG_FP64_HIERARCHY | v.VPS_FLAG_FP32_HIERARCHY | v.VPS_FLAG_POST_SAME_ORDER)
        b = P.rhs_sine_modes(kap, co)
        x = P.new()
        row = {"degree": k, "level": lev, "n_dofs": P.n(),
               "paper": {"l2_error": l2_paper, "double": {"iterations": it64_p, "s": t64_p},
                         "mixed": {"iterations": itmx_p, "s": tmx_p}, "solver": "GMRES"}}
        for name, mode in (("double", v.VPS_SOLVE_FP64), ("mixed", v.VPS_SOLVE_MIXED)):
            P.pcg_solve(b, x, 1e-9, 100, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = P.pcg_solve(b, x, 1e-9, 100, mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[name] = {"iterations": st.iterations, "s": dt, "dof_per_s": P.n() / dt,
                         "true_rel_residual": st.true_rel_residual, "l2_error": P.l2_error_sine_modes(x, kap, uc)}
        row["speedup"] = row["double"]["s"] / row["mixed"]["s"]
        del b, x
        P.close()
        torch.cuda.empty_cache()
        rows.append(row)
    return rows


def solve_2d_q7_run(v, torch, reps=5):
    """2D Q7 on 512^2 cells (12.8M DoFs), manufactured solution sin(pi x) sin(pi y), mixed and FP64
    CG with the V-cycle of the bench step, to 1e-10: solve time with the rhs resident, iterations,
    true residual and L2 error of the discrete solution."""
    import synth
    kap, co = synth.manufactured_sine(2)
    uc = [c / (math.pi ** 2 * sum(q * q for q in kk)) for kk, c in zip(kap, co)]
    P = v.Problem(2, 7, 9, v.VPS_FLAG_FP64_HIERARCHY | v.VPS_FLAG_FP32_HIERARCHY | v.VPS_FLAG_POST_SAME_ORDER)
    b = P.rhs_sine_modes(kap, co)
    x = P.new()
    out = {"workload": "2D Poisson Q7, 512^2 cells, u = sin(pi x) sin(pi y), CG to 1e-10", "n_dofs": P.n()}
    for name, mode in (("mixed", v.VPS_SOLVE_MIXED), ("fp64", v.VPS_SOLVE_FP64)):
        P.pcg_solve(b, x, 1e-10, 100, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, st = P.pcg_solve(b, x, 1e-10, 100, mode)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        out[name] = {"ms": ms, "dof_per_s": P.n() / (ms / 1e3), "iterations": st.iterations,
                     "true_rel_residual": st.true_rel_residual, "l2_error": P.l2_error_sine_modes(x, kap, uc)}
    out["mixed_speedup"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    del b, x
    P.close()
    torch.cuda.empty_cache()
    return out


def fmg_run(v, torch, P, kap, co):
    """Full multigrid on the bench problem (right-hand side on every level), both precisions."""
    res = {}
    for name, dt_, eps in (("fp64", torch.float64, 1e-9), ("fp32", torch.float32, 1e-4)):
        bl = [P.rhs_sine_modes(kap, co, level=l, dtype=dt_) for l in range(1, P.L + 1)]
        x = P.new(dt_)
        P.fmg_solve(bl, x, eps=eps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            _, st = P.fmg_solve(bl, x, eps=eps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 3
        res[name] = {"eps": eps, "vcycles_after_nested_iteration": st.iterations, "rel_residual": st.rel_residual,
                     "ms": ms, "dof_per_s": P.n() / (ms / 1e3)}
    return res


def variants_run(v, torch, P, b, stream):
    """Colour-pass forms on the finest level (Table 6 analogue): the fused kernel, the Boundary
    kernel (Sec. 4.1.3), the Separate pair (residual kernel, then the local-solve kernel) and the
    fused kernel with its residual contractions on the matrix cores (FP32 only; in FP64 that mode
    runs the fused kernel), per colour pass averaged over the 8 colours, and the V-cycle with each
    form."""
    res = {}
    flags = v.VPS_FLAG_FP64_HIERARCHY | v.VPS_FLAG_FP32_HIERARCHY | v.VPS_FLAG_POST_SAME_ORDER
    for name, dt_ in (("fp32", torch.float32), ("fp64", torch.float64)):
        bb = b.to(dt_)
        xx = torch.zeros_like(bb)
        r = torch.empty_like(bb)
        row = {}
        for form, mode in (("fused", v.VPS_MULTIPLICATIVE), ("boundary", v.VPS_MULTIPLICATIVE_BOUNDARY),
                           ("separate", v.VPS_MULTIPLICATIVE_SEPARATE), ("mfma", v.VPS_MULTIPLICATIVE_MFMA)):
            row[form + "_colour_pass_us"] = 1e6 * event_time(lambda: [P.color_pass(bb, xx, c, mode) for c in range(8)],
                                                             stream, 5) / 8
        row["separate_residual_kernel_us"] = 1e6 * event_time(lambda: P.residual(bb, xx, r), stream, 20)
        row["separate_solve_kernel_us"] = 1e6 * event_time(lambda: [P.color_pass(r, xx, c, v.VPS_ADDITIVE)
                                                                    for c in range(8)], stream, 5) / 8
        for form, fl in (("boundary", v.VPS_FLAG_BOUNDARY_SMOOTHER), ("separate", v.VPS_FLAG_SEPARATE_SMOOTHER),
                         ("mfma", v.VPS_FLAG_MFMA_SMOOTHER)):
            Q = v.Problem(P.dim, P.degree, P.L, flags | fl | v.VPS_FLAG_NO_SOLVER)
            row[form + "_vcycle_ms"] = 1e3 * event_time(lambda: Q.vcycle(bb, xx), stream, 5)
            Q.close()
        row["fused_vcycle_ms"] = 1e3 * event_time(lambda: P.vcycle(bb, xx), stream, 5)
        res[name] = {k_: round(v_, 2) for k_, v_ in row.items()}
    return res


def cpu_info():
    """CPU model and the threads the oracle's BLAS runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = None
    try:
        import threadpoolctl
        threads = max((p["num_threads"] for p in threadpoolctl.threadpool_info()), default=None)
    except Exception:
        pass
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return model, threads, len(os.sched_getaffinity(0))


def cpu_baseline(N, vcycles_per_solve, reps=3):
    """The FP64 oracle (NumPy/SciPy) on a bounded sample of the same workload.

    Sample: one full oracle V-cycle (Alg. 1 with the bench's colour order: smoothing steps of
    global residuals and dense-LU patch solves on every level, operator, transfers, dense coarse
    solve) on 3D Q4 64^3, best of `reps`.  A solve of n CG iterations applies n V-cycles (one before
    the first iteration, one after every iteration but the converged last); the CG operator
    applications and vector updates are not counted, so the scaled figure is an upper bound for the
    oracle's solve throughput.
    """
    import numpy as np
    import synth
    from oracle import mesh, multigrid, rhs, smoother, transfer
    kap, co = synth.fourier_modes(D, seed=1)
    b = rhs.rhs_sine_modes(D, K, L, kap, co)
    # oracle set-up (patch factorisations, index maps, 1D matrices) before the clock
    for lev in range(2, L + 1):
        mesh.global_1d_matrices(K, lev)
        mesh.boundary_mask(D, K, lev)
        smoother._patch_lu(D, K, lev)
        for c in range(2 ** D):
            smoother._colour_index_arrays(D, K, lev, c)
    multigrid.coarse_solve(D, K, np.zeros(mesh.n1d(K, 1) ** D))
    transfer.restrict(D, K, 2, np.zeros(mesh.n1d(K, 2) ** D))
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        multigrid.vcycle(D, K, L, b, np.zeros_like(b), post_reverse=False)
        times.append(time.perf_counter() - t0)
    t = min(times)
    model, threads, affinity = cpu_info()
    return {"value": N / (t * vcycles_per_solve), "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": "one FP64 oracle V-cycle on 3D Q4 64^3 (best of %d: %.1f s), scaled to the %d V-cycles of "
                      "one solve (upper bound: the CG operator and vector work is not counted)"
                      % (reps, t, vcycles_per_solve),
            "vcycle_s": times, "cpu_model": model, "cpus_available": affinity,
            "note": "a plain correctness oracle, not a tuned CPU solver"}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2405_19004_amd as v
    import synth

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.copy_mib:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 4}))
        return
    if a.serve_only:
        print(json.dumps(serving_run(v, a.serve, max_active=a.serve_slots, closed_loop_only=not a.serve_replays)))
        return
    if a.quick_2d:
        print(json.dumps({"solve_2d_q7": solve_2d_q7_run(v, torch)}))
        return
    FL = v.VPS_FLAG_FP64_HIERARCHY | v.VPS_FLAG_FP32_HIERARCHY
    P = v.Problem(D, K, L, FL | v.VPS_FLAG_POST_SAME_ORDER)
    if a.kernels_only:
        kap, co = synth.fourier_modes(D, seed=1)
        for dt_ in (torch.float32, torch.float64):
            bb = P.rhs_sine_modes(kap, co, dtype=dt_)
            xx = torch.zeros_like(bb)
            for _ in range(2):
                for c in range(8):
                    P.color_pass(bb, xx, c)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "patches_per_colour": list(P.info().color_count)}))
        return
    N = P.n()
    kap, co = synth.fourier_modes(D, seed=1)
    b = P.rhs_sine_modes(kap, co)
    x = P.new()

    for _ in range(a.warmup):
        _, st = P.pcg_solve(b, x, RTOL, 100, v.VPS_SOLVE_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(a.steps):
        _, st = P.pcg_solve(b, x, RTOL, 100, v.VPS_SOLVE_MIXED)
        its.append(st.iterations)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / a.steps
    out = {"metric": "smoother+V-cycle DoF/s (3D Q4, FP64 vs mixed); served-solve p50/p99 latency",
           "value": N * a.steps / dt, "unit": "DoF/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "3D Poisson Q4, 64^3 cells (257^3 = 16974593 nodes), 16-mode Fourier rhs seed 1, "
                                  "mixed-precision V-cycle CG to 1e-8", "dim": D, "degree": K, "level": L,
                      "n_dofs": N, "rtol": RTOL, "parallelism": "single GPU"},
           "mixed_solve": {"iterations": its[-1], "true_rel_residual": st.true_rel_residual, "ms": ms,
                           "vcycle": "same colour order before and after the correction, flexible CG"}}
    if a.quick:
        print(json.dumps(out))
        return

    def timed_solve(prob, mode, reps=3):
        xx = prob.new()
        prob.pcg_solve(b, xx, RTOL, 100, mode)
        torch.cuda.synchronize()
        t0_ = time.perf_counter()
        for _ in range(reps):
            _, s_ = prob.pcg_solve(b, xx, RTOL, 100, mode)
        torch.cuda.synchronize()
        ms_ = 1e3 * (time.perf_counter() - t0_) / reps
        return xx, {"iterations": s_.iterations, "ms": ms_, "dof_per_s": N / (ms_ / 1e3),
                    "true_rel_residual": s_.true_rel_residual}

    # FP64 solve with the same V-cycle, and both precisions with the symmetric V-cycle
    x64, out["fp64_solve"] = timed_solve(P, v.VPS_SOLVE_FP64)
    Psym = v.Problem(D, K, L, FL)
    _, out["mixed_solve_symmetric_vcycle"] = timed_solve(Psym, v.VPS_SOLVE_MIXED)
    x64s, out["fp64_solve_symmetric_vcycle"] = timed_solve(Psym, v.VPS_SOLVE_FP64)
    Psym.close()
    out["mixed_vs_fp64_rel_diff"] = float((x - x64).norm() / x64.norm())
    out["mixed_vs_fp64_symmetric_rel_diff"] = float((x - x64s).norm() / x64s.norm())
    out["mixed_speedup"] = out["fp64_solve"]["ms"] / ms

    # smoothing step and V-cycle per precision (events on the problem's stream)
    per = {}
    for name, dt_ in (("fp64", torch.float64), ("fp32", torch.float32)):
        bb = b.to(dt_)
        xx = torch.zeros_like(bb)
        t_s = event_time(lambda: P.smoother_apply(bb, xx), stream, 10)
        t_v = event_time(lambda: P.vcycle(bb, xx), stream, 10)
        per[name] = {"smoothing_step_ms": 1e3 * t_s, "smoother_dof_per_s": N / t_s,
                     "vcycle_ms": 1e3 * t_v, "vcycle_dof_per_s": N / t_v}
    out["smoother_vcycle"] = per
    out["smoother_variants"] = variants_run(v, torch, P, b, stream)
    out["fmg"] = fmg_run(v, torch, P, kap, co)

    # roofline of the dominant kernel: the FP32 colour pass on the finest level.  Algorithmic work
    # per patch is the measurement model's (smoother_patch_flops / smoother_patch_min_words); the
    # binding roof is the one with the longer time at peak.
    info = P.info()
    bb = b.to(torch.float32)
    xx = torch.zeros_like(bb)
    launches = 8 * 10
    t_all = event_time(lambda: [P.color_pass(bb, xx, c) for c in range(8)], stream, 10) / 8
    patches = sum(info.color_count[c] for c in range(8)) / 8
    flops = smoother_patch_flops(D, K) * patches
    bytes_ = 4 * smoother_patch_min_words(D, K) * patches
    issued = colour_pass_issued_flops(D, K) * patches
    lds_bytes = colour_pass_lds_bytes_3d(K, 4, 5) * patches  # five patches per workgroup at this size
    traffic = None
    tf = os.path.join(ROOT, "profiles", "colour_pass_3d_q4_fp32_traffic.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("source_hash") == smoother_source_hash():  # counters describe this exact kernel source
            traffic = rec.get("bytes_per_launch")
    t_hbm, t_alu = bytes_ / PEAK_HBM, flops / PEAK_FP32
    common = {"kernel": "colour_pass_kernel<3,4,float,multiplicative,5 patches per workgroup (wide shape)>",
              "avg_launch_us": 1e6 * t_all, "patches_per_launch": patches,
              "algorithmic_flops_per_patch": smoother_patch_flops(D, K),
              "algorithmic_words_per_patch": smoother_patch_min_words(D, K),
              "algorithmic_bytes_per_launch": bytes_, "algorithmic_flops_per_launch": flops,
              "launches_timed": launches,
              "alu": {"achieved_tflops": flops / t_all / 1e12, "peak_tflops": PEAK_FP32 / 1e12,
                      "frac": flops / t_all / PEAK_FP32,
                      # the 157.3 TFLOP/s peak needs packed FP32 instructions, which this build does
                      # not emit; one FP32 FMA per lane and clock gives half of it
                      "peak_tflops_unpacked": PEAK_FP32 / 2e12, "frac_unpacked": 2 * flops / t_all / PEAK_FP32},
              "hbm": {"achieved_gbps": bytes_ / t_all / 1e9, "peak_gbps": PEAK_HBM / 1e9,
                      "frac": bytes_ / t_all / PEAK_HBM},
              "executed": {"flops_per_launch": issued, "tflops": issued / t_all / 1e12,
                           "note": "structural zeros of the 1D patch matrices skipped, eigenvector symmetry used"},
              "lds": {"achieved_tbps": lds_bytes / t_all / 1e12, "peak_tbps": PEAK_LDS / 1e12,
                      "frac": lds_bytes / t_all / PEAK_LDS, "bytes_per_launch": lds_bytes,
                      "bytes_per_clock_per_cu": LDS_BYTES_PER_CLK}}
    if t_hbm >= t_alu:
        out["roofline"] = dict(bound="hbm", achieved=bytes_ / t_all / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                               frac=bytes_ / t_all / PEAK_HBM, traffic=traffic, **common)
    else:
        out["roofline"] = dict(bound="alu", achieved=flops / t_all / 1e12, peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                               frac=flops / t_all / PEAK_FP32, traffic=traffic, **common)
    xz = torch.zeros_like(b)
    t64 = event_time(lambda: [P.color_pass(b, xz, c) for c in range(8)], stream, 5) / 8
    bytes64 = 8 * smoother_patch_min_words(D, K) * patches
    out["roofline_fp64_colour_pass"] = {"bound": "hbm" if bytes64 / PEAK_HBM >= flops / PEAK_FP64 else "alu",
                                        "avg_launch_us": 1e6 * t64,
                                        "hbm_gbps": bytes64 / t64 / 1e9, "hbm_frac": bytes64 / t64 / PEAK_HBM,
                                        "alu_tflops": flops / t64 / 1e12, "alu_frac": flops / t64 / PEAK_FP64}
    P.close()
    progress("headline solve, components and colour-pass roofline done")

    out["solve_2d_q7"] = solve_2d_q7_run(v, torch)
    progress("2D Q7 solves done")

    if a.serve > 0:
        out["serving"] = serving_run(v, a.serve, max_active=a.serve_slots)
        progress("serving run done (%d requests)" % a.serve)
    if not a.no_table7:
        out["table7"] = table7_run(v, torch)
        progress("Table 7 problems done")
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(N, its[-1])
        progress("CPU oracle baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
