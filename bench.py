"""Benchmark: whole scattering solves per second on one MI355X.

Headline workload: the 3-wavelength cube (30^3 hexahedra, 10 nodes per
wavelength) around a centred PEC cube of one wavelength, ABC on all outer
faces, one plane wave of seeded direction/polarisation, FP64 solve to a
relative residual of 1e-8 (87 186 complex unknowns, 729 182 3x3 blocks).

One step = the whole hot path with the inputs already in HBM: ingest,
numbering, block pattern, assembly (FP64 + complex64 values + Jacobi),
right-hand side, COCG solve, scatter of H to the grid.

Also printed on the same JSON line:
  at_1e6        the same steps to 1e-6 with the FP64, mixed (complex64
                vectors) and matrix-mixed (complex64 matrix, complex128
                vectors) solvers: solves/s, iterations, p50/p99 latency
  spmv_hbm      block SpMV bandwidth on the 60^3 PEC-sphere + dielectric
                shell matrix (845 MB complex128, 434 MB complex64: larger
                than the 256 MB Infinity Cache)
  batched       the 40^3 PEC-sphere workload with 64 right-hand sides as one
                FP64 batched solve to 1e-6 (RHS/s, SpMM time, GB/s and
                TFLOP/s), against single-RHS FP64 and matrix-mixed solves of
                the same waves
  planes        the mirror-symmetric 30^3 PEC-cube box solved whole and as
                its quarter with an antisymmetry and a symmetry plane (FP64
                to 1e-8): solves/s of each and the quarter's deviation
  serving       a Poisson stream of scattering requests (meshes n^3 with n in
                [10, serve_n_hi], 1-4 waves each) through the continuous-
                batching server in matrix-mixed and FP64 precision (each
                wave its own solve, and a request's waves batched), and the
                plain FP64 solver one request at a time, all to 1e-6:
                requests/s, RHS/s, p50/p99 latency from arrival
  roofline      the dominant kernel of the timed steps (the FP64 block SpMV
                fused with p^T A p), timed with HIP events around every
                launch in the timed region
  cpu_baseline  the CPU oracle on a bounded sample of the headline workload
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

# HBM traffic of the dominant kernel from two rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE; mean KiB per working dispatch of the FP64
# SpMV-dot on the headline workload), each scaled by what the same counter
# reads for the 1 GiB copy probe (1 GiB read + 1 GiB written) in the same
# run.  Valid only for the kernel source it was taken on: reported as null
# once that file changes.
MEASURED_TRAFFIC = {
    "kernel": "k_cocg_spmv_dot<double>",
    "source": "paper_0704_2344_amd/csrc/krylov_kernels.hip",
    "sha256": "cd072f4a672b6d11d9031dc700142d67d72c97f56a7b1106968b4250634fdad5",
    "fetch_kib": 55018.17, "write_kib": 1426.30,
    "copy_fetch_kib": 524299.84, "copy_write_kib": 1048576.03, "copy_bytes": 1 << 30,
}


def measured_traffic():
    """Bytes per launch of the dominant kernel, or None if its source has
    changed since the counters were taken."""
    import hashlib
    m = MEASURED_TRAFFIC
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


def serving_leg(ctx, F, W, n_requests, rate, n_hi):
    """Replay a Poisson request stream in real time through the server (two
    precisions, each wave its own solve, and with a request's waves batched)
    and through the plain FP64 solver one request at a time."""
    reqs = W.serving_stream(n_requests=n_requests, rate_per_s=rate, seed=46, n_lo=10, n_hi=n_hi, nrhs_hi=4)
    n_rhs = sum(len(r.waves) for r in reqs)
    out = {"workload": (f"{n_requests} requests of the seeded serving stream (Poisson, {rate:g}/s), meshes n^3 "
                        f"with n in [10, {n_hi}], 1-4 waves each ({n_rhs} right-hand sides), PEC box or sphere, "
                        f"k0 in [pi, 4 pi] at 10 nodes per wavelength, rtol 1e-6")}
    # warm the kernels and the allocator
    srv = F.Server(ctx)
    p0, w0 = reqs[0].problem, reqs[0].waves
    t = srv.submit(p0, w0, precision=F.FEMH_FP64, rtol=1e-6)
    srv.poll(t, len(w0), None, want_field=False)
    srv.close()
    for name, prec, batch in (("server_mixed_matrix", F.FEMH_MIXED_MATRIX, False),
                              ("server_fp64", F.FEMH_FP64, False),
                              ("server_mixed_matrix_batched", F.FEMH_MIXED_MATRIX, True),
                              ("server_fp64_batched", F.FEMH_FP64, True)):
        srv = F.Server(ctx, batch_rhs=batch)
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            d = t0 + r.arrival_s - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append(srv.submit(r.problem, r.waves, precision=prec, rtol=1e-6))
        bad = 0
        for r, tk in zip(reqs, tickets):
            st, _, _ = srv.poll(tk, len(r.waves), None, want_field=False)
            bad += st != F.FEMH_OK
        el = time.perf_counter() - t0
        rep = srv.report()
        srv.close()
        out[name] = {"requests_per_s": rep["requests_per_second"], "rhs_per_s": rep["rhs_per_second"],
                     "p50_s": rep["p50_seconds"], "p99_s": rep["p99_seconds"], "failed": bad,
                     "wall_s": el, "peak_resident_bytes": rep["peak_resident_bytes"]}
    # plain FP64 solver, one request at a time in arrival order
    import torch
    lat = []
    bad = 0
    t0 = time.perf_counter()
    first = None
    for r in reqs:
        d = t0 + r.arrival_s - time.perf_counter()
        if d > 0:
            time.sleep(d)
        if first is None:
            first = time.perf_counter()
        P = F.Problem(ctx, r.problem)
        o = torch.zeros(P.grid_shape(len(r.waves)), dtype=torch.complex128, device="cuda")
        _, st = P.solve_dev(r.waves, o, precision=F.FEMH_FP64, rtol=1e-6)
        torch.cuda.synchronize()
        P.close()
        bad += st != F.FEMH_OK
        lat.append(time.perf_counter() - (t0 + r.arrival_s))
    span = time.perf_counter() - first
    out["plain_fp64_sequential"] = {"requests_per_s": n_requests / span, "rhs_per_s": n_rhs / span,
                                    "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                                    "failed": bad}
    plain = out["plain_fp64_sequential"]["rhs_per_s"]
    out["server_mixed_vs_plain_fp64"] = out["server_mixed_matrix"]["rhs_per_s"] / plain
    out["server_mixed_batched_vs_plain_fp64"] = out["server_mixed_matrix_batched"]["rhs_per_s"] / plain
    return out


def cpu_baseline(prob, waves, iters_needed, sample_iters):
    """The oracle as it stands (assembly + RHS + COCG), on a bounded sample:
    the full assembly and RHS, then `sample_iters` COCG iterations; the solve
    is extrapolated to `iters_needed` iterations."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, solve

    with threadpool_limits(1):
        t0 = time.perf_counter()
        A = fem.assemble(prob)
        t1 = time.perf_counter()
        b = fem.rhs(prob, waves)[:, 0]
        t2 = time.perf_counter()
        solve.cocg(A, b, rtol=1e-300, maxiter=sample_iters)
        t3 = time.perf_counter()
    per_iter = (t3 - t2) / sample_iters
    total = (t1 - t0) + (t2 - t1) + iters_needed * per_iter
    return {"value": 1.0 / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"full oracle assembly ({t1 - t0:.2f} s) and RHS ({t2 - t1:.3f} s) of the headline workload, "
                       f"then {sample_iters} FP64 COCG-Jacobi iterations ({per_iter * 1e3:.1f} ms each), "
                       f"extrapolated to the {iters_needed} iterations of the GPU FP64 solve; one thread")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cmp-steps", type=int, default=3, help="steps per solver in the 1e-6 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg but the headline")
    ap.add_argument("--extras", default="cmp,hbm,batched,planes,serving",
                    help="legs after the headline, comma-separated subset of cmp,hbm,batched,planes,serving")
    ap.add_argument("--batched-singles", type=int, default=4,
                    help="single-RHS solves per precision timed beside the batched leg (0 skips them)")
    ap.add_argument("--cpu-sample-iters", type=int, default=300)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run the 1 GiB copy probe (the denominator of the traffic scale factor)")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-n-hi", type=int, default=40)
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
    prob, waves = W.pec_cube(30)
    arrays = {"eps_r": torch.from_numpy(np.ascontiguousarray(prob.eps_r.reshape(-1))).to(dev),
              "mu_r": torch.from_numpy(np.ascontiguousarray(prob.mu_r.reshape(-1))).to(dev),
              "pec": torch.from_numpy(np.ascontiguousarray(prob.pec.reshape(-1))).to(dev)}
    out = torch.zeros((1, prob.nz + 1, prob.ny + 1, prob.nx + 1, 3), dtype=torch.complex128, device=dev)
    info = {}

    def step(precision, rtol):
        P = F.Problem(ctx, prob, device_arrays=arrays)
        stats, st = P.solve_dev(waves, out, precision=precision, rtol=rtol)
        if st != F.FEMH_OK:
            raise RuntimeError(f"solve failed: {stats}")
        info.update(nn=P.n_nodes, nnzb=P.nnzb, n=P.n_unknowns)
        P.close()
        return stats[0]

    def timed(precision, rtol, steps):
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

    for _ in range(args.warmup):
        step(F.FEMH_FP64, 1e-8)

    # ---- timed headline steps; the library brackets every eighth product
    # with HIP events on the solver's stream (a live sample of the timed region)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    value, elapsed, lat, st64 = timed(F.FEMH_FP64, 1e-8, args.steps)
    sec, cnt = ctx.profile_read(reset=True)
    ctx.profile(False)
    nn, nnzb = info["nn"], info["nnzb"]
    b128 = spmv_bytes(nn, nnzb, 16, 16)
    avg = sec[0] / max(cnt[0], 1)
    achieved = b128 / avg / 1e9

    traffic = measured_traffic()
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
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": ("pec_cube_30: 3-wavelength cube, 30^3 hexahedra, centred PEC cube of one "
                                "wavelength, ABC outer faces, one seeded plane wave, FP64 COCG-Jacobi to 1e-8; "
                                f"{info['n']} complex unknowns, {nnzb} 3x3 blocks"),
                   "global_batch": 1, "parallelism": "single GPU"},
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "solve": {"iters": st64["iters"], "restarts": st64["outer_iters"], "rel_residual": st64["rel_residual"],
                  "solve_s": st64["seconds"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "traffic_over_algorithmic": traffic / b128 if traffic else None,
                     "kernel": "k_cocg_spmv_dot<double> (complex128 block SpMV w = A z + z^T w)",
                     "bytes_per_launch": b128, "avg_launch_s": avg, "launches": cnt[0],
                     "timing": "HIP events around every 8th product of the timed solves",
                     "note": "the 111 MB complex128 matrix fits the 256 MB Infinity Cache"},
    }

    if args.copy_probe:
        result["copy_probe_GBps"] = ctx.bw_probe(1 << 30, 3)

    legs = set() if args.no_extras else {x for x in args.extras.split(",") if x}
    unknown = legs - {"cmp", "hbm", "batched", "planes", "serving"}
    if unknown:
        raise SystemExit(f"unknown --extras legs: {sorted(unknown)}")

    if "cmp" in legs:
        cmp = {}
        for name, prec in (("fp64", F.FEMH_FP64), ("mixed", F.FEMH_MIXED), ("mixed_matrix", F.FEMH_MIXED_MATRIX)):
            step(prec, 1e-6)
            sps, el, lt, s = timed(prec, 1e-6, args.cmp_steps)
            cmp[name] = {"solves_per_s": sps, "iters": s["iters"], "updates": s["outer_iters"],
                         "rel_residual": s["rel_residual"], "p50_s": float(np.percentile(lt, 50)),
                         "p99_s": float(np.percentile(lt, 99))}
        cmp["best_mixed_vs_fp64"] = max(cmp["mixed"]["solves_per_s"], cmp["mixed_matrix"]["solves_per_s"]) / \
            cmp["fp64"]["solves_per_s"]
        result["at_1e6"] = cmp

    if "hbm" in legs:
        # block SpMV on a matrix larger than the Infinity Cache
        p2, _ = W.pec_sphere_shell(60)
        P2 = F.Problem(ctx, p2)
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

    if "serving" in legs and args.serve_requests > 0:
        result["serving"] = serving_leg(ctx, F, W, args.serve_requests, args.serve_rate, args.serve_n_hi)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(prob, waves, st64["iters"], args.cpu_sample_iters)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
