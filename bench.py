"""Benchmark: scattering solves per second on one MI355X, mixed precision
against FP64 at an FP64 relative residual of 1e-6.

Headline workload (pec_sphere_shell_60): a 6-wavelength box of 60^3
hexahedra (10 nodes per wavelength) around a staircased PEC sphere of radius
1.5 wavelengths wrapped in a 0.3-wavelength dielectric shell (eps_r drawn
from U[2, 4] per element), ABC on the outer faces, one seeded plane wave:
644 136 complex unknowns, 5 561 948 3x3 blocks (845 MB of complex128 values,
434 MB complex64, both larger than the 256 MB Infinity Cache).  One step is
the whole hot path with the inputs already in HBM: ingest, numbering, block
pattern, assembly (FP64 + complex64 values + Jacobi), right-hand side, the
Krylov solve to an FP64 true residual of 1e-6, scatter of H to the grid.
`value` is the best mixed-precision mode (the complex64 matrix inside FP64
COCG with reliable updates against the FP64 matrix); the same steps in FP64
and the complex64-vector mode are timed beside it.

Also on the same JSON line:
  roofline      the dominant kernel of the headline steps (the complex64-matrix
                block SpMV fused with p^T A p), timed live with HIP events on
                the solver's stream
  pec_cube_30   the 30^3 PEC-cube workload (87 186 unknowns) in FP64 to 1e-8,
                with its own SpMV roofline (its 111 MB matrix is cache-resident)
  spmv_hbm      block SpMV bandwidth on the headline matrix in every precision
  batched       the 40^3 PEC sphere with 64 right-hand sides as one batch
  planes        the mirror-symmetric 30^3 box whole and as its quarter
  serving       the seeded request stream through the continuous-batching
                server at 0.5, 0.8 and 1.0 of its measured capacity, FP64
                and matrix-mixed, beside the plain FP64 solver
  cpu_baseline  the CPU oracle on a bounded sample of the headline workload,
                one thread and all threads, with the host CPU model
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E datasheet

# HBM traffic of the dominant kernels from two rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE; mean KiB per working dispatch of the kernel
# on the named workload), each scaled by what the same counter reads for the
# 1 GiB copy probe (1 GiB read + 1 GiB written) in the same run.  Valid only
# for the kernel source it was taken on: reported as null once that file
# changes.
MEASURED_TRAFFIC = {
    "m32_sphere_shell_60": {
        "kernel": "k_cocg_spmv_dot<double, float2>", "source": "paper_0704_2344_amd/csrc/krylov_kernels.hip",
        "sha256": "ffa42cb1b3bf8ff9da2ad9e716f922cfdb9ab6d3cde3b9b1bc086cc8969dd63a",
        "fetch_kib": 225810.49, "write_kib": 10129.70,
        "copy_fetch_kib": 524291.47, "copy_write_kib": 1048576.03, "copy_bytes": 1 << 30,
    },
    "c128_sphere_shell_60": {
        "kernel": "k_cocg_spmv_dot<double, double2>", "source": "paper_0704_2344_amd/csrc/krylov_kernels.hip",
        "sha256": "ffa42cb1b3bf8ff9da2ad9e716f922cfdb9ab6d3cde3b9b1bc086cc8969dd63a",
        "fetch_kib": 423813.98, "write_kib": 10150.82,
        "copy_fetch_kib": 524291.47, "copy_write_kib": 1048576.03, "copy_bytes": 1 << 30,
    },
}


def measured_traffic(key):
    """Bytes per launch of a dominant kernel, or None if no counters were
    taken for it or its source has changed since."""
    import hashlib
    m = MEASURED_TRAFFIC.get(key)
    if m is None:
        return None
    with open(os.path.join(ROOT, m["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != m["sha256"]:
            return None
    fetch_scale = m["copy_bytes"] / (m["copy_fetch_kib"] * 1024)
    write_scale = m["copy_bytes"] / (m["copy_write_kib"] * 1024)
    return m["fetch_kib"] * 1024 * fetch_scale + m["write_kib"] * 1024 * write_scale


def spmv_bytes(nn, nnzb, val_bytes, vec_bytes):
    """Algorithmic bytes of one block SpMV: every 3x3 block (9 complex values
    + one int32 column index) read once, the row pointers, x read once and y
    written once."""
    return nnzb * (9 * val_bytes + 4) + 4 * (nn + 1) + 2 * 3 * nn * vec_bytes


def spmm_bytes(nn, nnzb, ncols, s_val=16):
    """Algorithmic bytes of one batched SpMM: the matrix (s_val bytes per
    complex value) and its column indices read once, the row pointers, the
    complex128 directions read once and the complex128 products written
    once, for ncols columns."""
    return nnzb * (9 * s_val + 4) + 4 * (nn + 1) + 3 * nn * ncols * (16 + 16)


SERVE_MODES = {
    # name: (precision, batch a request's waves, inner_rtol (0 = the solver default))
    "fp64_batched": ("FEMH_FP64", True, 0.0),
    "mixed_matrix_batched": ("FEMH_MIXED_MATRIX", True, 0.0),
    "fp64": ("FEMH_FP64", False, 0.0),
    "mixed_matrix": ("FEMH_MIXED_MATRIX", False, 0.0),
    "mixed_matrix_batched_inner1e-5": ("FEMH_MIXED_MATRIX", True, 1e-5),
    "mixed_matrix_inner1e-5": ("FEMH_MIXED_MATRIX", False, 1e-5),
}


def fifo_finish_times(arrivals, service):
    """Finish times of a one-at-a-time server taking requests in arrival
    order: finish_i = max(arrival_i, finish_(i-1)) + service_i."""
    fin = np.zeros(len(arrivals))
    prev = 0.0
    for i, (a, s) in enumerate(zip(arrivals, service)):
        prev = max(float(a), prev) + float(s)
        fin[i] = prev
    return fin


def _replay(F, ctx, reqs, arrivals, prec, batch, inner, label):
    """Submit each request at its arrival time (seconds after the start),
    then wait for all; the server's report gives latency percentiles."""
    srv = F.Server(ctx, batch_rhs=batch)
    t0 = time.perf_counter()
    tickets = []
    for r, a in zip(reqs, arrivals):
        d = t0 + a - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets.append(srv.submit(r.problem, r.waves, precision=prec, rtol=1e-6, inner_rtol=inner))
    bad = []
    for i, (r, tk) in enumerate(zip(reqs, tickets)):
        st, _, stats = srv.poll(tk, len(r.waves), None, want_field=False)
        if st != F.FEMH_OK:
            bad.append({"request": i, "n": r.problem.nx, "waves": len(r.waves), "status": st,
                        "iters": [s["iters"] for s in stats], "rel_residual": [s["rel_residual"] for s in stats]})
        log(f"  {label}: request {i + 1}/{len(reqs)} (n = {r.problem.nx}, {len(r.waves)} waves) done at "
            f"{time.perf_counter() - t0:.2f} s")
    el = time.perf_counter() - t0
    rep = srv.report()
    srv.close()
    n_rhs = sum(len(r.waves) for r in reqs)
    return {"wall_s": el, "requests_per_s": len(reqs) / el, "rhs_per_s": n_rhs / el,
            "p50_s": rep["p50_seconds"], "p99_s": rep["p99_seconds"], "failed": len(bad), "failures": bad,
            "peak_resident_bytes": rep["peak_resident_bytes"]}


def serving_leg(ctx, F, W, n_requests, n_lo, n_hi, nrhs_hi, loads, modes, capacity=None):
    """The seeded serving stream through the continuous-batching server.

    Capacity is measured first: every request submitted at once to the FP64
    server (each request's waves batched), requests/s over the whole span.
    Then the same requests arrive as a Poisson stream at each load (a
    fraction of that capacity, in requests/s) in real time, through each
    server mode; every mode sees the same arrival times, so latency and
    throughput compare at equal offered traffic.  The plain FP64 solver (one
    request at a time: assembly, solve, field to host) is timed once per
    request; its latencies at each load follow from those service times by
    the first-in-first-out recursion finish_i = max(arrival_i, finish_(i-1))
    + service_i, which is what a one-at-a-time solver does.  With no loads,
    every mode gets the all-at-once run instead (its own capacity)."""
    import torch

    unknown = set(modes) - set(SERVE_MODES) - {"plain_fp64"}
    if unknown:
        raise SystemExit(f"unknown --serve-modes: {sorted(unknown)}")
    reqs = W.serving_stream(n_requests=n_requests, rate_per_s=1.0, seed=46, n_lo=n_lo, n_hi=n_hi, nrhs_hi=nrhs_hi)
    unit = np.array([r.arrival_s for r in reqs])     # arrivals of a rate-1 Poisson stream
    n_rhs = sum(len(r.waves) for r in reqs)
    unk = [3 * (r.problem.nx + 1) ** 3 for r in reqs]
    out = {"workload": (f"{n_requests} requests of the seeded serving stream: meshes n^3 with n in [{n_lo}, {n_hi}] "
                        f"(up to {max(unk)} grid unknowns), PEC box or sphere, k0 in [pi, 4 pi] at 10 nodes per "
                        f"wavelength, 1-{nrhs_hi} waves each ({n_rhs} right-hand sides), FP64 relative residual "
                        f"1e-6; " + ("Poisson arrivals at each load's rate" if loads else "all submitted at once")),
           "loads": list(loads)}
    # warm the kernels and the allocator on a small request
    pw, ww = W.serving_request(np.random.default_rng(7), n_lo=10, n_hi=12, nrhs_hi=2)
    for batch in (True, False):
        srv = F.Server(ctx, batch_rhs=batch)
        t = srv.submit(pw, ww, precision=F.FEMH_FP64, rtol=1e-6)
        srv.poll(t, len(ww), None, want_field=False)
        srv.close()
    if capacity is None and loads:
        sat = _replay(F, ctx, reqs, np.zeros(n_requests), F.FEMH_FP64, True, 0.0, "capacity (fp64_batched, all at once)")
        capacity = sat["requests_per_s"]
        out["saturated_fp64_batched"] = sat
    out["capacity_requests_per_s"] = capacity
    for name in modes:
        if name == "plain_fp64":
            continue
        pn, batch, inner = SERVE_MODES[name]
        if not loads:
            out[f"saturated_{name}"] = _replay(F, ctx, reqs, np.zeros(n_requests), getattr(F, pn), batch, inner,
                                               f"{name}, all at once")
            continue
        res = {}
        for load in loads:
            res[f"load_{load:g}"] = _replay(F, ctx, reqs, unit / (load * capacity), getattr(F, pn), batch, inner,
                                            f"{name} at {load:g}x capacity")
        out[f"server_{name}"] = res
    if "plain_fp64" in modes:
        service = []
        for i, r in enumerate(reqs):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            P = F.Problem(ctx, r.problem)
            o = torch.zeros(P.grid_shape(len(r.waves)), dtype=torch.complex128, device="cuda")
            _, st = P.solve_dev(r.waves, o, precision=F.FEMH_FP64, rtol=1e-6)
            o.cpu()
            P.close()
            service.append(time.perf_counter() - s0)
            log(f"  plain fp64: request {i + 1}/{len(reqs)} (n = {r.problem.nx}, {len(r.waves)} waves) "
                f"{service[-1]:.3f} s")
        service = np.array(service)
        res = {"service_s_total": float(service.sum()), "capacity_requests_per_s": n_requests / service.sum()}
        for load in loads:
            arr = unit / (load * capacity)
            fin = fifo_finish_times(arr, service)
            lat = fin - arr
            res[f"load_{load:g}"] = {"wall_s": float(fin[-1]), "rhs_per_s": n_rhs / float(fin[-1]),
                                     "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99))}
        out["plain_fp64_sequential"] = res
    # throughput of each server mode against the plain solver on the same
    # arrivals at the highest load
    if loads and "plain_fp64_sequential" in out:
        top = f"load_{max(loads):g}"
        plain = out["plain_fp64_sequential"][top]["rhs_per_s"]
        for name in modes:
            if name != "plain_fp64" and f"server_{name}" in out:
                out[f"server_{name}_vs_plain_fp64"] = out[f"server_{name}"][top]["rhs_per_s"] / plain
    return out


def log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, waves, iters_needed, sample_iters, threads):
    """The oracle as it stands (assembly + RHS + COCG), on a bounded sample:
    the full assembly and RHS, then `sample_iters` COCG iterations; the solve
    is extrapolated to `iters_needed` iterations.  threads = None lets the
    numerical libraries use every core."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, solve

    with threadpool_limits(threads):
        t0 = time.perf_counter()
        A = fem.assemble(prob)
        t1 = time.perf_counter()
        b = fem.rhs(prob, waves)[:, 0]
        t2 = time.perf_counter()
        solve.cocg(A, b, rtol=1e-300, maxiter=sample_iters)
        t3 = time.perf_counter()
    per_iter = (t3 - t2) / sample_iters
    total = (t1 - t0) + (t2 - t1) + iters_needed * per_iter
    return {"value": 1.0 / total, "unit": "solves/s", "assembly_s": t1 - t0, "rhs_s": t2 - t1,
            "per_iter_s": per_iter, "sample_iters": sample_iters}


def spmv_event_roofline(ctx_slot_sec, ctx_slot_cnt, nn, nnzb, val_bytes, vec_bytes, kernel, key, note):
    avg = ctx_slot_sec / max(ctx_slot_cnt, 1)
    nbytes = spmv_bytes(nn, nnzb, val_bytes, vec_bytes)
    achieved = nbytes / avg / 1e9
    traffic = measured_traffic(key)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
            "traffic_over_algorithmic": traffic / nbytes if traffic else None,
            "kernel": kernel, "bytes_per_launch": nbytes, "avg_launch_s": avg, "launches": ctx_slot_cnt,
            "timing": "HIP events on the solver's stream around every 8th product of the timed solves",
            "note": note}


def bic_apply_bytes(n, nnz_l, rows_per_block):
    """Algorithmic bytes of one block incomplete Cholesky application: the
    factor once per sweep (L with its diagonal, U without: 16-byte value and
    4-byte column per entry, 4-byte row starts), 1 / l_uu once per sweep, r
    read twice (the start and the closing dot products), z written once."""
    nnz_u = nnz_l - n
    nblk = -(-n // rows_per_block)
    return 20 * (nnz_l + nnz_u) + 8 * (n + 1) + 2 * 16 * n + 3 * 16 * n + 64 * nblk


def bicp_leg(ctx, F, W, torch, dev, with_sphere, blocks=(4, 16, 64)):
    """FP64 COCG with Jacobi against block incomplete Cholesky (blocks of B
    nodes) on the 30^3 PEC cube to 1e-8 (and the 60^3 coated sphere to 1e-6
    when asked): iterations, solve time, time per iteration, and the
    application alone (femh_bic0_apply_dev, HIP events).  Each solve runs
    twice; the first includes building the factor."""
    cases = [("pec_cube_30", W.pec_cube(30), 1e-8,
              "30^3 hexahedra, centred PEC cube of one wavelength, ABC outer faces, one seeded wave")]
    if with_sphere:
        cases.append(("pec_sphere_shell_60", W.pec_sphere_shell(60), 1e-6,
                      "60^3 hexahedra, PEC sphere with a lossy dielectric shell, one seeded wave"))
    out = {}
    for name, (prob, waves), rtol, what in cases:
        P = F.Problem(ctx, prob)
        o = torch.zeros(P.grid_shape(1), dtype=torch.complex128, device=dev)
        leg = {"workload": f"{name}: {what}; FP64 COCG to {rtol:g}; {P.n_unknowns} unknowns, {P.nnzb} blocks"}
        rv = torch.randn(P.n_unknowns, dtype=torch.complex128, device=dev)
        zv = torch.zeros_like(rv)
        runs = [("jacobi", {})] + [(f"bic0_{b}", dict(precond=F.FEMH_PRECOND_BIC0, precond_block=b)) for b in blocks]
        for tag, kw in runs:
            times = []
            for _ in range(2):
                torch.cuda.synchronize()
                a = time.perf_counter()
                st, stc = P.solve_dev(waves, o, precision=F.FEMH_FP64, rtol=rtol, **kw)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - a)
            s0 = st[0]
            r = {"status": stc, "iters": s0["iters"], "restarts": s0["outer_iters"], "rel_residual": s0["rel_residual"],
                 "solve_s": times[1], "us_per_iter": times[1] / max(s0["iters"], 1) * 1e6,
                 "first_solve_s": times[0]}
            if tag != "jacobi":
                nodes = kw["precond_block"]
                _, col, _ = P.export_bic0(nodes)
                t_apply = P.bic0_apply_dev(rv, zv, nodes, reps=20)
                nbytes = bic_apply_bytes(P.n_unknowns, len(col), 3 * nodes)
                r.update({"factor_entries": len(col), "apply_us": t_apply * 1e6, "apply_bytes": nbytes,
                          "apply_GBps": nbytes / t_apply / 1e9,
                          "time_vs_jacobi": times[1] / leg["jacobi"]["solve_s"]})
            leg[tag] = r
            log(f"  bicp {name} {tag}: {s0['iters']} iterations, {times[1]:.3f} s"
                + (f", apply {r['apply_us']:.1f} us" if "apply_us" in r else ""))
        out[name] = leg
        P.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed headline steps (mixed precision)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cmp-steps", type=int, default=2,
                    help="timed FP64 steps beside the headline (0 skips FP64 and the complex64-vector solve)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg but the headline")
    ap.add_argument("--extras", default="cube,hbm,batched,planes,bicp,serving",
                    help="legs after the headline, comma-separated subset of cube,hbm,batched,planes,bicp,serving")
    ap.add_argument("--bicp-sphere", action="store_true",
                    help="bicp leg: also the 60^3 coated sphere (about a minute of solves)")
    ap.add_argument("--cube-steps", type=int, default=10)
    ap.add_argument("--batched-singles", type=int, default=2,
                    help="single-RHS solves per precision timed beside the batched leg (0 skips them)")
    ap.add_argument("--cpu-sample-iters", type=int, default=60)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run the 1 GiB copy probe (the denominator of the traffic scale factor)")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-n-lo", type=int, default=10, help="smallest mesh n of the serving requests")
    ap.add_argument("--serve-n-hi", type=int, default=26, help="largest mesh n of the serving requests")
    ap.add_argument("--serve-nrhs-hi", type=int, default=16)
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0",
                    help="offered loads, fractions of the measured capacity ('' = each mode all at once)")
    ap.add_argument("--serve-modes", default="fp64_batched,mixed_matrix_batched,plain_fp64",
                    help="comma-separated subset of " + ",".join(list(SERVE_MODES) + ["plain_fp64"]))
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="requests/s to take as the capacity instead of measuring it (0 = measure)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}); the multi-GPU path is a design "
              f"only and is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_0704_2344_amd import femh as F

    dev = torch.device("cuda", 0)
    ctx = F.Context(0)

    def resident(prob):
        return {"eps_r": torch.from_numpy(np.ascontiguousarray(prob.eps_r.reshape(-1))).to(dev),
                "mu_r": torch.from_numpy(np.ascontiguousarray(prob.mu_r.reshape(-1))).to(dev),
                "pec": torch.from_numpy(np.ascontiguousarray(prob.pec.reshape(-1))).to(dev)}

    def make_step(prob, waves, arrays, info):
        out = torch.zeros((len(waves), prob.nz + 1, prob.ny + 1, prob.nx + 1, 3), dtype=torch.complex128,
                          device=dev)

        def step(precision, rtol, allow_fail=False):
            P = F.Problem(ctx, prob, device_arrays=arrays)
            stats, st = P.solve_dev(waves, out, precision=precision, rtol=rtol, max_iter=100000)
            info.update(nn=P.n_nodes, nnzb=P.nnzb, n=P.n_unknowns)
            P.close()
            if st != F.FEMH_OK and not allow_fail:
                raise RuntimeError(f"solve failed: {stats}")
            return stats[0]
        return step

    def timed(step, precision, rtol, steps):
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for _ in range(steps):
            s0 = time.perf_counter()
            last = step(precision, rtol)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
        el = time.perf_counter() - t0
        return steps / el, el, lat, last

    # ---- headline: the 60^3 coated sphere, matrix-mixed vs FP64 to 1e-6
    prob, waves = W.pec_sphere_shell(60)
    info = {}
    step = make_step(prob, waves, resident(prob), info)
    log(f"headline pec_sphere_shell_60: {args.warmup} warm-up + {args.steps} timed matrix-mixed steps")
    for _ in range(args.warmup):
        step(F.FEMH_MIXED_MATRIX, 1e-6)
    # timed steps; the library brackets every eighth product with HIP events
    # on the solver's stream (a live sample of the timed region)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    value, elapsed, lat, st_m = timed(step, F.FEMH_MIXED_MATRIX, 1e-6, args.steps)
    sec, cnt = ctx.profile_read(reset=True)
    nn, nnzb = info["nn"], info["nnzb"]
    fp_sps, fp_lat, st_f, st_c64, t_c64 = None, [float("nan")], None, None, None
    sec64, cnt64 = [0.0] * 4, [0] * 4
    if args.cmp_steps > 0:
        log(f"matrix-mixed {value:.3f} solves/s; {args.cmp_steps} FP64 steps")
        fp_sps, fp_el, fp_lat, st_f = timed(step, F.FEMH_FP64, 1e-6, args.cmp_steps)
        sec64, cnt64 = ctx.profile_read(reset=True)
        log(f"FP64 {fp_sps:.3f} solves/s; one complex64-vector solve")
        # the complex64-vector mode, once (it breaks down on this system)
        t0 = time.perf_counter()
        st_c64 = step(F.FEMH_MIXED, 1e-6, allow_fail=True)
        t_c64 = time.perf_counter() - t0
    ctx.profile(False)

    result = {
        "metric": "block SpMV GB/s (% HBM peak); solves/s + p99 latency at 1e-6, mixed vs FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 matrix, f64 vectors and sums",
        "data": "synthetic",
        "config": {"workload": ("pec_sphere_shell_60: 60^3 hexahedra (6 wavelengths, 10 nodes per wavelength), "
                                "staircased PEC sphere of radius 1.5 wavelengths in a dielectric shell "
                                "(eps_r ~ U[2,4]), ABC outer faces, one seeded plane wave; matrix-mixed COCG-Jacobi "
                                f"to an FP64 relative residual of 1e-6; {info['n']} complex unknowns, "
                                f"{nnzb} 3x3 blocks"),
                   "global_batch": 1, "parallelism": "single GPU"},
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "solve": {"iters": st_m["iters"], "reliable_updates": st_m["outer_iters"],
                  "rel_residual": st_m["rel_residual"], "solve_s": st_m["seconds"]},
        "fp64": None if st_f is None else {
            "solves_per_s": fp_sps, "p50_s": float(np.percentile(fp_lat, 50)),
            "p99_s": float(np.percentile(fp_lat, 99)), "steps": args.cmp_steps, "iters": st_f["iters"],
            "rel_residual": st_f["rel_residual"]},
        "mixed_vs_fp64": value / fp_sps if fp_sps else None,
        "mixed_c64_vectors": None if st_c64 is None else {
            "status": st_c64["status"], "iters": st_c64["iters"], "rel_residual": st_c64["rel_residual"],
            "seconds": t_c64},
        "roofline": spmv_event_roofline(sec[3], cnt[3], nn, nnzb, 8, 16,
                                        "k_cocg_spmv_dot<double, float2> (complex64 block values, complex128 "
                                        "vectors, FP64 sums: q = A p and p^T q)", "m32_sphere_shell_60",
                                        "434 MB complex64 matrix, larger than the 256 MB Infinity Cache"),
        "roofline_fp64_product": None if not cnt64[0] else spmv_event_roofline(sec64[0], cnt64[0], nn, nnzb, 16, 16,
                                                     "k_cocg_spmv_dot<double> (complex128 block SpMV w = A z "
                                                     "+ z^T w)", "c128_sphere_shell_60",
                                                     "845 MB complex128 matrix"),
    }

    if args.copy_probe:
        result["copy_probe_GBps"] = ctx.bw_probe(1 << 30, 3)

    legs = set() if args.no_extras else {x for x in args.extras.split(",") if x}
    unknown = legs - {"cube", "hbm", "batched", "planes", "bicp", "serving"}
    if unknown:
        raise SystemExit(f"unknown --extras legs: {sorted(unknown)}")

    if "cube" in legs:
        log("leg cube")
    if "cube" in legs:
        # the 30^3 PEC cube, FP64 to 1e-8 (cache-resident matrix)
        pc, wc = W.pec_cube(30)
        ic = {}
        stepc = make_step(pc, wc, resident(pc), ic)
        stepc(F.FEMH_FP64, 1e-8)
        ctx.profile(True)
        ctx.profile_read(reset=True)
        sps, el, lt, sc = timed(stepc, F.FEMH_FP64, 1e-8, args.cube_steps)
        sec_c, cnt_c = ctx.profile_read(reset=True)
        ctx.profile(False)
        result["pec_cube_30"] = {
            "workload": ("pec_cube_30: 30^3 hexahedra, centred PEC cube of one wavelength, ABC outer faces, one "
                         f"seeded wave, FP64 COCG-Jacobi to 1e-8; {ic['n']} unknowns, {ic['nnzb']} blocks"),
            "solves_per_s": sps, "p50_s": float(np.percentile(lt, 50)), "p99_s": float(np.percentile(lt, 99)),
            "iters": sc["iters"], "rel_residual": sc["rel_residual"],
            "roofline": spmv_event_roofline(sec_c[0], cnt_c[0], ic["nn"], ic["nnzb"], 16, 16,
                                            "k_cocg_spmv_dot<double>", "c128_pec_cube_30",
                                            "the 111 MB complex128 matrix fits the 256 MB Infinity Cache")}

    if "hbm" in legs:
        log("leg hbm")
    if "hbm" in legs:
        # block SpMV on the headline matrix (larger than the Infinity Cache)
        P2 = F.Problem(ctx, prob)
        n2 = P2.n_unknowns
        x = torch.randn(n2, dtype=torch.complex128, device=dev)
        y = torch.zeros_like(x)
        x32 = x.to(torch.complex64)
        y32 = torch.zeros_like(x32)
        hb = {}
        for name, prec, xx, yy, vb, xb in (("c128", F.FEMH_FP64, x, y, 16, 16),
                                           ("c64", F.FEMH_MIXED, x32, y32, 8, 8),
                                           ("c64_matrix_c128_vectors", F.FEMH_MIXED_MATRIX, x, y, 8, 16)):
            P2.spmv_dev(xx, yy, prec, reps=3)
            t = P2.spmv_dev(xx, yy, prec, reps=20)
            gb = spmv_bytes(P2.n_nodes, P2.nnzb, vb, xb) / t / 1e9
            hb[name] = {"us": t * 1e6, "GBps": gb, "frac_hbm_peak": gb / HBM_PEAK_GBPS}
        # the symmetric half store (storage #1 analogue): same product, about
        # half the stored blocks
        t_half = P2.spmv_half_dev(x, y, reps=3)
        t_half = P2.spmv_half_dev(x, y, reps=10)
        hb["c128_half_store"] = {"us": t_half * 1e6, "vs_full_store": hb["c128"]["us"] / (t_half * 1e6)}
        hb["workload"] = f"pec_sphere_shell_60 matrix: {n2} unknowns, {P2.nnzb} blocks"
        hb["copy_probe_GBps"] = ctx.bw_probe(1 << 30, 10)
        result["spmv_hbm"] = hb
        P2.close()
    if "batched" in legs:
        log("leg batched")
    if "batched" in legs:
        # batched right-hand sides
        p3, w3 = W.pec_sphere_batched(40)
        P3 = F.Problem(ctx, p3)
        o3 = torch.zeros(P3.grid_shape(64), dtype=torch.complex128, device=dev)
        # nine columns take the wide layout: tunes its SpMM, warms the graph path
        P3.solve_dev(w3[:9], o3[:9], batched=True, precision=F.FEMH_FP64, rtol=1e-3)
        torch.cuda.synchronize()
        a = time.perf_counter()
        stats3, st3 = P3.solve_dev(w3, o3, batched=True, precision=F.FEMH_FP64, rtol=1e-6)
        torch.cuda.synchronize()
        el3 = time.perf_counter() - a
        its = [s["iters"] for s in stats3]
        # the solver's SpMM (same kernel and grid), timed on its own
        Xs = torch.randn(P3.n_unknowns, 64, dtype=torch.complex128, device=dev)
        Ys = torch.zeros(P3.n_unknowns, 64, dtype=torch.complex128, device=dev)
        t_spmm = P3.spmm_dev(Xs, Ys, reps=20, precision=F.FEMH_FP64)
        del Xs, Ys
        flops = P3.nnzb * 9 * 64 * 8
        # single-RHS solves of the first waves (matrix-mixed and plain FP64), for comparison
        o1 = torch.zeros(P3.grid_shape(1), dtype=torch.complex128, device=dev)
        ns = args.batched_singles
        single = {"mixed_matrix": None, "fp64": None}
        for name, prec in (("mixed_matrix", F.FEMH_MIXED_MATRIX), ("fp64", F.FEMH_FP64)):
            if ns <= 0:
                break
            torch.cuda.synchronize()
            a = time.perf_counter()
            for wv in w3[:ns]:
                P3.solve_dev([wv], o1, precision=prec, rtol=1e-6)
            torch.cuda.synchronize()
            single[name] = (time.perf_counter() - a) / ns
        result["batched"] = {"workload": "pec_sphere_40_b64: 40^3, PEC sphere R=1 wavelength, 64 RHS, to 1e-6",
                             "matrix": "complex128",
                             "status": st3, "rhs_per_s": 64 / el3, "seconds": el3,
                             "iters_min": min(its), "iters_max": max(its),
                             "max_rel_residual": max(s["rel_residual"] for s in stats3),
                             "spmm_tile": P3.spmm_tile(), "spmm_us": t_spmm * 1e6,
                             "spmm_GBps": spmm_bytes(P3.n_nodes, P3.nnzb, 64) / t_spmm / 1e9,
                             "spmm_TFLOPs": flops / t_spmm / 1e12,
                             "single_rhs_mixed_matrix_rhs_per_s":
                                 1.0 / single["mixed_matrix"] if single["mixed_matrix"] else None,
                             "single_rhs_fp64_rhs_per_s": 1.0 / single["fp64"] if single["fp64"] else None,
                             "speedup_vs_single_fp64": (64 / el3) * single["fp64"] if single["fp64"] else None}
        P3.close()

    if "planes" in legs:
        log("leg planes")
    if "planes" in legs:
        # symmetry planes: the mirror-symmetric 30^3 box against its quarter
        # (antisymmetry plane on -x, symmetry plane on -y)
        n4 = 30
        legs_out = {}
        fields = {}
        for name, cx in (("whole", False), ("quarter", True)):
            p4, w4 = W.mirrored_pec_cube(n4, side=1.0, cut_x=cx, cut_y=cx)
            o4 = torch.zeros((1, p4.nz + 1, p4.ny + 1, p4.nx + 1, 3), dtype=torch.complex128, device=dev)
            P4 = F.Problem(ctx, p4)
            P4.solve_dev(w4, o4, precision=F.FEMH_FP64, rtol=1e-8)        # warm-up
            torch.cuda.synchronize()
            a = time.perf_counter()
            reps4 = 3
            for _ in range(reps4):
                s4, st4 = P4.solve_dev(w4, o4, precision=F.FEMH_FP64, rtol=1e-8)
            torch.cuda.synchronize()
            t4 = (time.perf_counter() - a) / reps4
            legs_out[name] = {"status": st4, "n_unknowns": P4.n_unknowns, "iters": s4[0]["iters"],
                              "solve_s": t4, "solves_per_s": 1.0 / t4}
            fields[name] = o4[0].cpu().numpy()
            P4.close()
        ref = fields["whole"][:, n4 // 2:, n4 // 2:, :]
        legs_out["quarter_vs_whole_rel_l2"] = float(np.linalg.norm(fields["quarter"] - ref) / np.linalg.norm(ref))
        legs_out["speedup"] = legs_out["quarter"]["solves_per_s"] / legs_out["whole"]["solves_per_s"]
        legs_out["workload"] = ("mirrored_pec_cube_30: 30^3 box centred on a PEC cube of one wavelength, x-polarised "
                                "wave along +z, FP64 to 1e-8; the quarter x >= 0, y >= 0 with n x H = 0 on x = 0 "
                                "and n . H = 0 on y = 0")
        result["planes"] = legs_out

    if "bicp" in legs:
        log("leg bicp")
        result["bicp"] = bicp_leg(ctx, F, W, torch, dev, args.bicp_sphere)

    if "serving" in legs:
        log("leg serving")
    if "serving" in legs and args.serve_requests > 0:
        result["serving"] = serving_leg(ctx, F, W, args.serve_requests, args.serve_n_lo, args.serve_n_hi,
                                        args.serve_nrhs_hi, [float(x) for x in args.serve_loads.split(",") if x],
                                        [x for x in args.serve_modes.split(",") if x],
                                        args.serve_capacity or None)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one thread, then all threads)")
        one = cpu_baseline(prob, waves, st_m["iters"], args.cpu_sample_iters, 1)
        ncpu = os.cpu_count() or 1
        allc = cpu_baseline(prob, waves, st_m["iters"], args.cpu_sample_iters, None)
        best = allc if allc["value"] >= one["value"] else one
        result["cpu_baseline"] = {
            "value": best["value"], "unit": "solves/s", "cores": ncpu if best is allc else 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": ncpu,
            "one_core": one, "all_cores": allc,
            "sample": (f"the oracle's full assembly and RHS of the headline workload, then {args.cpu_sample_iters} "
                       f"FP64 COCG-Jacobi iterations, extrapolated to the {st_m['iters']} iterations of the GPU "
                       f"matrix-mixed solve; run once on one thread and once with every core available to the "
                       f"numerical libraries (SciPy's sparse product is single-threaded either way)")}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
