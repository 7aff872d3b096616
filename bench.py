"""Benchmark of the H-IDBF-LU hot path on one MI355X.

Workload (the timed one): Archimedean spiral r = a*theta, theta in [pi, 6 pi],
N = 2^20 segments at 10 per wavelength, 64 incident plane waves at uniform
angles, complex64 butterfly / leaf factors, leaf 64, ID tolerance 1e-6,
block-LU preconditioner, mixed-precision GMRES(30).

A timed step is one complete batched GMRES(30) cycle over the 64 right-hand
sides: the FP64 residual, 30 Arnoldi steps (each one preconditioner
application -- lower and upper block sweeps -- and one H-IDBF matvec, FP64
Gram-Schmidt, FP64 Givens), the least-squares update through one more
preconditioner application, and the FP64 refinement residual with the
complex64 factors.  `value` is the throughput of the H-IDBF-LU applications
inside those steps: their algorithmic bytes (every unit's factors,
permutations and descriptor once per application, plus 2 N-vectors per RHS)
over the wall time of the whole step, GMRES work included.

The spiral is a resonant scatterer: GMRES(30) does not reach 1e-6 there in a
bounded number of cycles (the paper observes the same weakening of the
preconditioner for spirals of more than one turn).  The seconds-per-RHS
comparison to relres <= 1e-6 (batched complex64 vs plain single-RHS
complex128) therefore runs on the semicircle at the same N = 2^20, where both
converge.

Beside it: the single-RHS complex64 matvec and preconditioner timed with HIP
events on the launch stream (the roofline figure), the autotuned execution
parameters, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the matvec at the default workload
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_stage_lanes_pipe_matvec_hbm_traffic_spiral_2p20_c64.txt")
METRIC = "H-IDBF-LU apply GB/s; s/RHS at N=2^20 batched c64 vs plain c128, relres≤1e-6"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources that decide what the single-RHS matvec reads and writes: the
# factor layout, the launch schedule and the stage kernel
MATVEC_SOURCES = ("hbf_internal.h", "kernels.h", "lane_unit.h", "plan.cpp", "ctx.cpp", "stage_pipe.hip",
                  "stage_lanes.hip")


def host_cores():
    """Worker processes for the CPU oracle: the cores this process may run
    on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def sources_digest():
    """sha256 over the single-RHS matvec's sources (name and contents, in
    name order): identifies the build a set of hardware-counter readings was
    taken on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1901_11371_amd", "csrc")
    for name in sorted(MATVEC_SOURCES):
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per matvec launch from the committed counter summary, if its
    readings were taken on these very sources (else None)."""
    import re
    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    src = re.search(r"sources sha256: ([0-9a-f]{64})", text)
    tb = re.search(r"traffic bytes per launch: (\d+)", text)
    if not src or not tb or src.group(1) != sources_digest():
        return None
    return int(tb.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--no-srhs", action="store_true", help="skip the semicircle seconds-per-RHS comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--mode", default="full", choices=["full", "matvec", "precond", "precond_batch", "matvec_batch", "scale", "iterations", "profile",
                             "counters"],
                    help="matvec / precond: only the single-RHS apply loop; precond_batch: the nrhs-RHS "
                         "preconditioner loop with the autotuned parameters (for profiling)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--srhs-geometry", default="semicircle", choices=["semicircle", "spiral"],
                    help="geometry of the seconds-per-RHS comparison")
    ap.add_argument("--srhs-n", type=int, default=0, help="N of the seconds-per-RHS comparison (0: --n)")
    ap.add_argument("--method", default="gmres", choices=["gmres", "tfqmr"],
                    help="Krylov method of the seconds-per-RHS and scale solves")
    ap.add_argument("--superleaf", type=int, default=0,
                    help="log2 leaves per exactly inverted diagonal block of the sweeps (0: library default)")
    ap.add_argument("--params", default=None,
                    help="JSON object of execution parameters to set instead of autotuning (profiling modes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; multi-GPU execution is not part of this library "
              "(the path would shard by right-hand sides)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1901_11371_amd import autotune, inputs
    from paper_1901_11371_amd.hbf import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.mode == "scale":
        scale_workload(args)
        return
    if args.mode == "iterations":
        iteration_counts(args)
        return
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    n, R, m = args.n, args.nrhs, args.restart
    wl = inputs.workload(2, n=n, nrhs=R)
    log(f"[bench] building spiral N={n} (host construction + upload)")
    t0 = time.time()
    ctx = Context(wl.curves, inputs.KAPPA, wl.n0, wl.tol, dtype="c64", max_nrhs=R, restart=m,
                  superleaf=args.superleaf, verbose=True)
    t_build = time.time() - t0
    st = ctx.stats
    log(f"[bench] built in {t_build:.1f}s: mean rank {st['mean_rank']:.2f} max {st['max_rank']} "
        f"butterfly {st['bytes_butterfly']/1e9:.2f} GB dense {st['bytes_dense']/1e9:.2f} GB")
    elt = 8
    vec1 = 2 * n * elt
    mv_fac = st["apply_bytes_matvec"] - vec1   # factors + permutations + descriptors
    pc_fac = st["apply_bytes_precond"] - vec1

    def timed_loop(fn, reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    if args.params:
        for k, v in json.loads(args.params).items():
            ctx.tune(k, v)
    x1 = torch.tensor(inputs.random_complex(n, 7), dtype=torch.complex64, device=dev)
    if args.mode in ("profile", "counters"):
        # for rocprofv3: a plain copy of known size (the counter calibration
        # kernel), the single-RHS matvec, then the 64-RHS matvec and (profile
        # only) the preconditioner, each kernel identifiable by name.  The
        # counter passes use "counters": no preconditioner, so no kernel runs
        # from a HIP graph while counters are collected.
        big = torch.empty(1 << 27, dtype=torch.complex64, device=dev)
        big2 = torch.empty_like(big)
        big2.copy_(big)
        torch.cuda.synchronize()
        del big, big2
        t1 = timed_loop(lambda: ctx.matvec(x1), args.reps)
        XB = torch.tensor(inputs.random_complex((R, n), 8), dtype=torch.complex64, device=dev)
        tb = timed_loop(lambda: ctx.matvec(XB), 3)
        out = {"mode": args.mode, "matvec_1rhs_ms": t1 * 1e3, f"matvec_{R}rhs_ms": tb * 1e3,
               "launches_matvec": st["launches_matvec"], "apply_bytes_matvec": st["apply_bytes_matvec"]}
        if args.mode == "profile":
            out[f"precond_{R}rhs_ms"] = timed_loop(lambda: ctx.precond(XB), 2) * 1e3
        print(json.dumps(out))
        return
    if args.mode == "matvec":
        # a plain copy of known size first: the calibration kernel for the HBM counters
        big = torch.empty(1 << 27, dtype=torch.complex64, device=dev)
        big2 = torch.empty_like(big)
        big2.copy_(big)
        torch.cuda.synchronize()
        del big, big2
    t_mv = timed_loop(lambda: ctx.matvec(x1), args.reps)
    mv_launches = st["launches_matvec"]
    log(f"[bench] 1-RHS c64 matvec {t_mv*1e3:.3f} ms ({mv_launches} launches) -> "
        f"{(mv_fac + vec1)/t_mv/1e9:.1f} GB/s")
    if args.mode == "matvec":
        print(json.dumps({"mode": "matvec", "ms": t_mv * 1e3, "gbs": (mv_fac + vec1) / t_mv / 1e9,
                          "launches": mv_launches, "avg_launch_us": t_mv / mv_launches * 1e6}))
        return
    if args.mode == "matvec_batch":
        XB = torch.tensor(inputs.random_complex((R, n), 8), dtype=torch.complex64, device=dev)
        t_mb = timed_loop(lambda: ctx.matvec(XB), max(2, args.reps // 4))
        print(json.dumps({"mode": "matvec_batch", "nrhs": R, "ms": t_mb * 1e3}))
        return
    if args.mode == "precond_batch":
        if not args.params:
            autotune.apply(ctx, R) or autotune.autotune(ctx, nrhs=R, reps=1)
        XB = torch.tensor(inputs.random_complex((R, n), 8), dtype=torch.complex64, device=dev)
        t_pb = timed_loop(lambda: ctx.precond(XB), max(2, args.reps // 10))
        print(json.dumps({"mode": "precond_batch", "nrhs": R, "ms": t_pb * 1e3}))
        return
    t_pc = timed_loop(lambda: ctx.precond(x1), max(2, args.reps // 10))
    log(f"[bench] 1-RHS c64 preconditioner {t_pc*1e3:.3f} ms -> {(pc_fac + vec1)/t_pc/1e9:.1f} GB/s")
    if args.mode == "precond":
        print(json.dumps({"mode": "precond", "ms": t_pc * 1e3, "gbs": (pc_fac + vec1) / t_pc / 1e9}))
        return

    tuned = None
    if not args.no_tune:
        t0 = time.time()
        tuned = autotune.apply(ctx, R)
        if tuned is None:
            tuned = {"params": autotune.autotune(ctx, nrhs=R, reps=1, verbose=False)}
        log(f"[bench] tuned parameters for nrhs={R}: {tuned['params']} ({time.time()-t0:.1f}s)")

    B = torch.tensor(inputs.plane_wave_rhs(wl.curves, wl.angles), dtype=torch.complex128, device=dev)

    def cycle():
        return ctx.solve(B, tol=1e-6, restart=m, max_iters=m)

    for w in range(args.warmup):
        log(f"[bench] warmup cycle {w}")
        cycle()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        X, infos, status = cycle()
        log(f"[bench] step {k}: iters {max(i['iters'] for i in infos)} "
            f"max relres {max(i['relres'] for i in infos):.2e}")
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    iters = max(i["iters"] for i in infos)
    relres = [i["relres"] for i in infos]
    # applications per cycle: one matvec and one preconditioner per Arnoldi step, one
    # preconditioner for the update and one FP64-vector residual matvec
    n_pc = iters + 1
    n_mv = iters
    bytes_step = (n_mv * (mv_fac + 2 * n * R * elt) + n_pc * (pc_fac + 2 * n * R * elt)
                  + (mv_fac + 2 * n * R * 16))
    value = bytes_step / t_step / 1e9
    log(f"[bench] GMRES({m}) cycle on {R} RHS: {t_step:.3f} s, apply {value:.1f} GB/s, "
        f"relres max {max(relres):.2e} median {float(np.median(relres)):.2e}")

    # batched apply timings (HIP events on the launch stream)
    XR = torch.tensor(inputs.random_complex((R, n), 8), dtype=torch.complex64, device=dev)
    t_mvR = timed_loop(lambda: ctx.matvec(XR), 3)
    t_pcR = timed_loop(lambda: ctx.precond(XR), 2)
    log(f"[bench] {R}-RHS matvec {t_mvR*1e3:.2f} ms, preconditioner {t_pcR*1e3:.2f} ms")
    x_spiral0 = X[0].cpu().numpy()
    b_spiral0 = B[0].cpu().numpy()
    ctx.close()
    del X, B, XR
    torch.cuda.empty_cache()

    srhs = None
    if not args.no_srhs:
        srhs = seconds_per_rhs(args.srhs_geometry, args.srhs_n or n, R, m, args.method)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl.curves, x_spiral0, b_spiral0, mv_fac + vec1)

    mv_gbs = (mv_fac + vec1) / t_mv / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded analytic curves, plane-wave excitations)",
        "config": {"workload": f"archimedean spiral N={n}, {R} plane waves, complex64 factors, leaf 64, "
                               f"ID tol 1e-6, one batched GMRES({m}) cycle per step",
                   "n": n, "nrhs": R, "restart": m},
        "step": {"gmres_iters": iters, "matvecs": n_mv + 1, "precond_applies": n_pc,
                 "bytes": bytes_step, "relres_max": max(relres), "relres_median": float(np.median(relres))},
        "s_per_rhs": srhs,
        "apply": {"matvec_1rhs_ms": t_mv * 1e3, "precond_1rhs_ms": t_pc * 1e3,
                  f"matvec_{R}rhs_ms": t_mvR * 1e3, f"precond_{R}rhs_ms": t_pcR * 1e3,
                  "matvec_bytes_1rhs": mv_fac + vec1, "precond_bytes_1rhs": pc_fac + vec1,
                  "precond_1rhs_gbs": (pc_fac + vec1) / t_pc / 1e9},
        "roofline": {"bound": "hbm", "kernel": "single-RHS H-IDBF matvec stage launches (k_stage_lanes for stages of small units, k_stage_pipe for the rest)",
                     "achieved": round(mv_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(mv_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if n == (1 << 20) else None,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "launches_per_apply": mv_launches,
                     "avg_launch_us": round(t_mv / mv_launches * 1e6, 3)},
        "tuned": tuned["params"] if tuned else None,
        "build": {"host_seconds": t_build, "mean_rank": st["mean_rank"], "max_rank": st["max_rank"],
                  "bytes_butterfly": st["bytes_butterfly"], "bytes_dense": st["bytes_dense"],
                  "bytes_precond": st["bytes_precond"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def seconds_per_rhs(geometry, n, R, m, method):
    """A batched complex64 solve of R plane waves vs the plain single-RHS
    complex128 solve on the same geometry, both to relres <= 1e-6."""
    import torch

    from paper_1901_11371_amd import autotune, inputs
    from paper_1901_11371_amd.hbf import Context
    dev = torch.device("cuda", 0)
    curves = inputs.semicircle(n) if geometry == "semicircle" else inputs.archimedean_spiral(n)
    angles = inputs.uniform_angles(R)
    B = torch.tensor(inputs.plane_wave_rhs(curves, angles), dtype=torch.complex128, device=dev)
    max_iters = 500 if geometry == "semicircle" else 20000
    t0 = time.time()
    ctx = Context(curves, inputs.KAPPA, 64, 1e-6, dtype="c64", max_nrhs=R, restart=m, cache_plan=True)
    log(f"[bench] {geometry} N={n} complex64 context built in {time.time()-t0:.1f}s")
    tuned_b = autotune.apply(ctx, R) or {"params": autotune.autotune(ctx, nrhs=R, reps=2)}
    log(f"[bench] {geometry} batched parameters: {tuned_b['params']}")
    kw = dict(tol=1e-6, max_iters=max_iters, method=method)
    ctx.solve(B, **dict(kw, max_iters=4))   # warm-up: captures the step and sweep graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, infos, _ = ctx.solve(B, **kw)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    x0 = X[0].clone()
    ctx.close()
    del X
    torch.cuda.empty_cache()
    t0 = time.time()
    ctx128 = Context(curves, inputs.KAPPA, 64, 1e-6, dtype="c128", max_nrhs=1, restart=m, cache_plan=True)
    log(f"[bench] {geometry} complex128 context built in {time.time()-t0:.1f}s (host plan reused)")
    tuned_p = autotune.apply(ctx128, 1) or {"params": autotune.autotune(ctx128, nrhs=1, reps=2)}
    log(f"[bench] {geometry} plain parameters: {tuned_p['params']}")
    b0 = B[0].contiguous()
    ctx128.solve(b0, **dict(kw, max_iters=4))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x128, info128, _ = ctx128.solve(b0, **kw)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx128.close()
    diff = float(torch.linalg.norm(x0 - x128) / torch.linalg.norm(x128))
    out = {"workload": f"{geometry} N={n}, {R} plane waves, relres 1e-6, {method}",
           "batched_c64": t_batched / R, "plain_c128": t_plain,
           "speedup": t_plain / (t_batched / R),
           "batched_iters_max": max(i["iters"] for i in infos),
           "batched_relres_max": max(i["relres"] for i in infos),
           "batched_converged": all(i["converged"] for i in infos),
           "plain_iters": info128[0]["iters"], "plain_relres": info128[0]["relres"],
           "plain_converged": info128[0]["converged"],
           "batched_params": tuned_b["params"], "plain_params": tuned_p["params"],
           "batched_c64_vs_c128_solution_rel_diff": diff}
    log(f"[bench] s/RHS {geometry}: batched c64 {t_batched/R*1e3:.2f} ms, plain c128 {t_plain*1e3:.1f} ms, "
        f"iterations {out['batched_iters_max']} / {out['plain_iters']}, solution diff {diff:.2e}")
    return out


def scale_workload(args):
    """The scale workload: 8 disjoint strips and arcs (random lengths and
    orientations), N = 2^22, 256 plane waves solved in chunks of 64 with
    complex64 factors and FP64 refinement to relres 1e-6; matvec parity on
    sampled exact rows first."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from oracle import efie
    from paper_1901_11371_amd import inputs
    from paper_1901_11371_amd.hbf import Context
    n = args.n if args.n != (1 << 20) else (1 << 22)
    nrhs_total, chunk = 256, 64
    wl = inputs.workload(4, n=n, nrhs=nrhs_total)
    dev = torch.device("cuda", 0)
    log(f"[scale] building {wl.curves.ncurves} curves N={n} (host construction + upload)")
    t0 = time.time()
    ctx = Context(wl.curves, inputs.KAPPA, wl.n0, wl.tol, dtype="c64", max_nrhs=chunk, restart=args.restart,
                  verbose=True)
    t_build = time.time() - t0
    st = ctx.stats
    log(f"[scale] built in {t_build:.1f}s: mean rank {st['mean_rank']:.2f} max {st['max_rank']} "
        f"butterfly {st['bytes_butterfly']/1e9:.2f} GB dense {st['bytes_dense']/1e9:.2f} GB "
        f"leaf inverses {st['bytes_precond']/1e9:.2f} GB workspace {st['bytes_workspace']/1e9:.2f} GB")
    # matvec parity on sampled rows (oracle, one process per core)
    rho, w = efie.segments(wl.curves.xy, wl.curves.node_off)
    cores = host_cores()
    rows = np.sort(np.random.default_rng(inputs.SEED_BASE + 4).choice(n, 2 * cores, replace=False))
    X = inputs.random_complex((2, n), 54)
    Y = ctx.matvec(torch.tensor(X, dtype=torch.complex64, device=dev)).cpu().numpy()
    t0 = time.perf_counter()
    parts = np.array_split(rows, cores)
    with mp.get_context("spawn").Pool(cores) as pool:
        outs = pool.map(_oracle_rows, [(p, X.T, rho, w, inputs.KAPPA) for p in parts])
    ref = np.concatenate(outs).T
    err = float(np.linalg.norm(Y[:, rows] - ref) / np.linalg.norm(ref))
    log(f"[scale] matvec sampled rel err {err:.3e} ({len(rows)} rows, oracle {time.perf_counter()-t0:.1f}s)")
    # apply timings
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps
    x1 = torch.tensor(X[0], dtype=torch.complex64, device=dev)
    t_mv1 = timed(lambda: ctx.matvec(x1), 5)
    XB = torch.tensor(inputs.random_complex((chunk, n), 55), dtype=torch.complex64, device=dev)
    t_mvb = timed(lambda: ctx.matvec(XB), 2)
    t_pcb = timed(lambda: ctx.precond(XB), 1)
    del XB
    log(f"[scale] matvec 1 RHS {t_mv1*1e3:.2f} ms, {chunk} RHS {t_mvb*1e3:.1f} ms; preconditioner {chunk} RHS "
        f"{t_pcb*1e3:.1f} ms")
    # 256 RHS in chunks of 64
    infos = []
    t_solve = 0.0
    for c0 in range(0, nrhs_total, chunk):
        B = torch.tensor(inputs.plane_wave_rhs(wl.curves, wl.angles[c0:c0 + chunk]), dtype=torch.complex128,
                         device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, status = ctx.solve(B, tol=1e-6, max_iters=2000, method=args.method)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_solve += dt
        infos += info
        log(f"[scale] RHS {c0}..{c0 + chunk - 1}: {dt:.1f}s, iters max {max(i['iters'] for i in info)}, "
            f"relres max {max(i['relres'] for i in info):.2e}, status {status}")
        del B
    ctx.close()
    out = {"mode": "scale", "workload": f"{wl.curves.ncurves} strips/arcs N={n}, {nrhs_total} plane waves in "
                                        f"chunks of {chunk}, complex64 factors, relres 1e-6, {args.method}",
           "n": n, "build_s": t_build, "matvec_sampled_rel_err": err, "sampled_rows": len(rows),
           "matvec_1rhs_ms": t_mv1 * 1e3, f"matvec_{chunk}rhs_ms": t_mvb * 1e3,
           f"precond_{chunk}rhs_ms": t_pcb * 1e3,
           "solve_s_per_rhs": t_solve / nrhs_total, "iters_max": max(i["iters"] for i in infos),
           "relres_max": max(i["relres"] for i in infos), "converged": all(i["converged"] for i in infos),
           "bytes_butterfly": st["bytes_butterfly"], "bytes_dense": st["bytes_dense"],
           "bytes_precond": st["bytes_precond"], "mean_rank": st["mean_rank"], "max_rank": st["max_rank"]}
    print(json.dumps(out), flush=True)


def iteration_counts(args):
    """Iteration counts with and without the preconditioner over the
    families of the paper's iteration study (Sec. 4): N (semicircle), arc
    angle, Archimedean-spiral rotation and arc-array size; one plane wave at
    pi/6, complex128 factors and vectors, relres 1e-6."""
    import math

    import torch

    from paper_1901_11371_amd import inputs
    from paper_1901_11371_amd.hbf import Context
    dev = torch.device("cuda", 0)
    n = 1 << 14
    method = args.method
    cap = 3000
    fams = {
        "N (semicircle)": [(f"N={k}", inputs.semicircle(k)) for k in (1 << 12, 1 << 13, 1 << 14, 1 << 15, 1 << 16)],
        "arc angle": [(f"angle={a / math.pi:.2f}pi", inputs.arc_with_angle(n, a))
                      for a in (math.pi / 4, math.pi / 2, math.pi, 1.5 * math.pi, 1.9 * math.pi)],
        "spiral rotation": [(f"rotation={r / math.pi:.0f}pi", inputs.archimedean_spiral(n, math.pi, math.pi + r))
                            for r in (math.pi, 2 * math.pi, 3 * math.pi, 4 * math.pi, 5 * math.pi)],
        "arc array": [(f"count={k}", inputs.arc_array(n, k)) for k in (1, 2, 4, 8, 16)],
    }
    out = {"mode": "iterations", "method": method, "tol": 1e-6, "cap": cap, "families": {}}
    for fam, members in fams.items():
        rows = []
        for label, c in members:
            b = torch.tensor(inputs.plane_wave_rhs(c, [math.pi / 6])[0], device=dev)
            row = {"member": label, "n": c.n_segments}
            for prec in ("block", "none"):
                ctx = Context(c, inputs.KAPPA, 64, 1e-6, dtype="c128", prec=prec, max_nrhs=1, restart=100)
                t0 = time.perf_counter()
                _, info, st = ctx.solve(b, tol=1e-6, restart=100, max_iters=cap, method=method)
                torch.cuda.synchronize()
                row[f"iters_{prec}"] = info[0]["iters"]
                row[f"converged_{prec}"] = bool(info[0]["converged"])
                row[f"seconds_{prec}"] = time.perf_counter() - t0
                ctx.close()
            log(f"[iterations] {fam} {label}: with the preconditioner {row['iters_block']}"
                f"{'' if row['converged_block'] else '+'} , without {row['iters_none']}"
                f"{'' if row['converged_none'] else '+'}")
            rows.append(row)
        out["families"][fam] = rows
    print(json.dumps(out), flush=True)


def _oracle_rows(args):
    """Worker: exact rows of A x with the oracle (one process per core)."""
    rows, x, rho, w, kappa = args
    from oracle import efie
    return efie.exact_rows_matvec(rows, x, rho, w, kappa, chunk=8)


def cpu_baseline(curves, x_gpu, b, mv_bytes, rows_per_core=12):
    """The CPU oracle as it stands, on the host's cores, on a bounded sample.

    * Matrix-free exact rows of A x (FP64, SciPy Hankel) for a seeded sample
      of rows of the spiral, one process per core, scaled by N / rows to one
      full apply and expressed in the H-IDBF matvec's algorithmic GB/s (the
      value).  As a by-product: the exact-operator residual of the GPU
      spiral iterate on the sampled rows.
    * The dense path at N = 4096 (the plain-strip workload): Z assembly,
      GEMV and LU factorisation + solve (NumPy / SciPy with the BLAS's own
      threads)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import efie
    from paper_1901_11371_amd import inputs
    cores = host_cores()
    rho, w = efie.segments(curves.xy, curves.node_off)
    n = rho.shape[0]
    rng = np.random.default_rng(inputs.SEED_BASE + 2)
    nrows = rows_per_core * cores
    rows = np.sort(rng.choice(n, nrows, replace=False))
    x = x_gpu.astype(np.complex128)
    parts = np.array_split(rows, cores)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        outs = pool.map(_oracle_rows, [(p, x, rho, w, inputs.KAPPA) for p in parts])
    t = time.perf_counter() - t0
    ax = np.concatenate(outs)
    t_full = t * n / nrows
    res = np.linalg.norm(b[rows] - ax) / np.linalg.norm(b[rows])
    log(f"[bench] oracle: {nrows} exact rows on {cores} cores in {t:.1f}s -> full apply {t_full:.0f}s "
        f"(extrapolated); sampled exact residual of the GPU iterate {res:.2e}")
    # dense path at N = 4096 (plain strip)
    wl = inputs.workload(0)
    rho4, w4 = efie.segments(wl.curves.xy, wl.curves.node_off)
    t0 = time.perf_counter()
    A4 = efie.dense_A(rho4, w4, inputs.KAPPA)
    t_asm = time.perf_counter() - t0
    b4 = inputs.plane_wave_rhs(wl.curves, wl.angles)[0]
    t0 = time.perf_counter()
    for _ in range(10):
        y4 = efie.matvec(A4, b4)
    t_gemv = (time.perf_counter() - t0) / 10
    t0 = time.perf_counter()
    x4 = efie.lu_solve(A4, b4)
    t_lu = time.perf_counter() - t0
    rr = float(efie.relres(A4, x4, b4))
    log(f"[bench] oracle dense N=4096: assembly {t_asm:.2f}s, GEMV {t_gemv*1e3:.1f} ms, LU solve {t_lu:.2f}s "
        f"(relres {rr:.1e})")
    del y4
    return {"value": round(mv_bytes / t_full / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{nrows} seeded rows of the exact matrix-free FP64 product A x at N={n}, one process per "
                      f"core ({cores}), {t:.1f} s, scaled by N/{nrows} to one apply; GB/s = the H-IDBF matvec's "
                      f"algorithmic bytes over that time",
            "seconds_per_apply_extrapolated": t_full,
            "gpu_iterate_sampled_exact_relres": float(res),
            "dense_4096": {"assembly_s": t_asm, "gemv_s": t_gemv, "lu_solve_s": t_lu, "relres": rr,
                           "workload": "plain strip N=4096, complex128, NumPy/SciPy BLAS threads"}}


if __name__ == "__main__":
    main()
