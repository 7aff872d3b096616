"""Benchmark of the H-IDBF-LU hot path on one MI355X.

Workload: Archimedean spiral r = a*theta, theta in [pi, 6 pi], N = 2^20
segments at 10 per wavelength, 64 incident plane waves at uniform angles,
complex64 butterfly / leaf factors, block-LU preconditioner, relres <= 1e-6
(FP64 residual, mixed-precision refinement).

A timed step is one batched solve of the 64 right-hand sides (every row of
the hot path: factor streaming, H-IDBF matvec, lower and upper block
sweeps, GMRES with FP64 Gram-Schmidt and Givens, FP64 refinement, batching).
`value` is the throughput of the H-IDBF-LU applications inside those solves:
algorithmic bytes of every matvec and preconditioner application / time.

Beside it: the 1-RHS complex64 apply measured with HIP events (roofline
figure), seconds per RHS of the batched complex64 solve vs the plain 1-RHS
complex128 solve, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain complex128 solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mode", default="full", choices=["full", "matvec", "precond", "solve"],
                    help="matvec/precond: only the 1-RHS apply loop (for profiling)")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it "
              "(the path would shard by right-hand sides, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1901_11371_amd import inputs
    from paper_1901_11371_amd.hbf import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    n = args.n
    R = args.nrhs
    kappa = inputs.KAPPA
    curves = inputs.archimedean_spiral(n)
    angles = inputs.uniform_angles(R)
    log(f"[bench] building spiral N={n} (host construction + upload)")
    t0 = time.time()
    ctx = Context(curves, kappa, 64, 1e-6, dtype="c64", max_nrhs=R, restart=30, cache_plan=not args.no_plain)
    t_build = time.time() - t0
    st = ctx.stats
    log(f"[bench] built in {t_build:.1f}s: mean rank {st['mean_rank']:.2f} max {st['max_rank']} "
        f"butterfly {st['bytes_butterfly']/1e9:.2f} GB dense {st['bytes_dense']/1e9:.2f} GB")
    elt = 8
    vec_bytes = 2 * n * elt
    mv_bytes = st["bytes_butterfly"] + st["bytes_dense"] + st["bytes_index"] + vec_bytes
    # a preconditioner application reads every off-diagonal block once (lower sweep: F21,
    # upper sweep: F12), the dense neighbour blocks, the leaf inverses and the vectors
    nl = n // 64
    diag_bytes = nl * 64 * 64 * elt
    pc_bytes = st["bytes_butterfly"] + (st["bytes_dense"] - diag_bytes) + st["bytes_precond"] \
        + st["bytes_index"] + 3 * vec_bytes

    stream = torch.cuda.current_stream(dev)

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

    x1 = torch.tensor(inputs.random_complex(n, 7), dtype=torch.complex64, device=dev)
    t_mv = timed_loop(lambda: ctx.matvec(x1), args.reps)
    log(f"[bench] 1-RHS c64 matvec {t_mv*1e3:.3f} ms -> {mv_bytes/t_mv/1e9:.1f} GB/s")
    if args.mode == "matvec":
        print(json.dumps({"mode": "matvec", "ms": t_mv * 1e3, "gbs": mv_bytes / t_mv / 1e9}))
        return
    t_pc = timed_loop(lambda: ctx.precond(x1), max(2, args.reps // 10))
    log(f"[bench] 1-RHS c64 preconditioner {t_pc*1e3:.3f} ms -> {pc_bytes/t_pc/1e9:.1f} GB/s")
    if args.mode == "precond":
        print(json.dumps({"mode": "precond", "ms": t_pc * 1e3, "gbs": pc_bytes / t_pc / 1e9}))
        return

    B = torch.tensor(inputs.plane_wave_rhs(curves, angles), dtype=torch.complex128, device=dev)
    for w in range(args.warmup):
        log(f"[bench] warmup solve {w}")
        ctx.solve(B, tol=1e-6)
    torch.cuda.synchronize()
    infos = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        X, infos, status = ctx.solve(B, tol=1e-6)
        log(f"[bench] step {k}: iters {max(i['iters'] for i in infos)} refinements {infos[0]['refinements']}"
            f" max relres {max(i['relres'] for i in infos):.2e}")
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / args.steps
    iters = max(i["iters"] for i in infos)
    refs = infos[0]["refinements"]
    relres = max(i["relres"] for i in infos)
    # applications per solve: one matvec and one preconditioner per GMRES iteration, one
    # preconditioner per cycle for the update and one FP64 residual matvec per refinement
    n_mv = iters + refs
    n_pc = iters + refs
    bytes_per_solve = n_mv * (mv_bytes - vec_bytes + 2 * n * R * elt) + n_pc * (pc_bytes - 3 * vec_bytes + 3 * n * R * elt)
    value = bytes_per_solve / t_solve / 1e9
    s_per_rhs = t_solve / R
    log(f"[bench] batched c64 solve {t_solve:.3f} s ({s_per_rhs*1e3:.2f} ms/RHS), apply {value:.1f} GB/s")

    plain = None
    if not args.no_plain:
        log("[bench] plain complex128 context (same geometry, 1 RHS)")
        ctx.close()
        torch.cuda.empty_cache()
        ctx128 = Context(curves, kappa, 64, 1e-6, dtype="c128", max_nrhs=1, restart=30)
        b0 = B[0].contiguous()
        ctx128.solve(b0, tol=1e-6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x128, info128, _ = ctx128.solve(b0, tol=1e-6)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        plain = {"s_per_rhs": t_plain, "iters": info128[0]["iters"], "relres": info128[0]["relres"]}
        err_vs_c128 = float(torch.linalg.norm(X[0] - x128) / torch.linalg.norm(x128))
        plain["batched_c64_vs_c128_rel_diff"] = err_vs_c128
        log(f"[bench] plain c128 solve {t_plain:.3f} s/RHS, iters {plain['iters']}, "
            f"c64-vs-c128 solution diff {err_vs_c128:.2e}")
        ctx128.close()
    else:
        ctx.close()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(curves, kappa, X[0].cpu().numpy(), B[0].cpu().numpy(), mv_bytes)

    line = {
        "metric": "H-IDBF-LU apply GB/s; s/RHS at N=2^20 batched c64 vs plain c128, relres<=1e-6",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_solve * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded analytic spiral, plane-wave excitations)",
        "config": {"workload": f"archimedean spiral N={n}, {R} plane waves, complex64 factors, leaf 64, "
                               f"ID tol 1e-6, GMRES(30) relres 1e-6",
                   "nrhs": R, "n": n},
        "s_per_rhs": {"batched_c64": s_per_rhs, "plain_c128": plain["s_per_rhs"] if plain else None},
        "solve": {"gmres_iters": iters, "refinements": refs, "max_relres": relres},
        "plain_c128": plain,
        "apply_1rhs_c64": {"matvec_ms": t_mv * 1e3, "matvec_gbs": mv_bytes / t_mv / 1e9,
                           "precond_ms": t_pc * 1e3, "precond_gbs": pc_bytes / t_pc / 1e9,
                           "matvec_bytes": mv_bytes, "precond_bytes": pc_bytes},
        "roofline": {"bound": "hbm", "achieved": round(mv_bytes / t_mv / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(mv_bytes / t_mv / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
        "build": {"host_seconds": t_build, "mean_rank": st["mean_rank"], "max_rank": st["max_rank"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(curves, kappa, x_gpu, b, mv_bytes):
    """The CPU oracle on a bounded sample: exact rows of A x (matrix-free FP64,
    SciPy Hankel) for a seeded sample of rows, timed on all host cores; scaled
    to one full apply.  As a by-product it reports the GPU solution's residual
    on the sampled rows."""
    import numpy as np

    from oracle import efie
    cores = os.cpu_count() or 1
    rho, w = efie.segments(curves.xy, curves.node_off)
    n = rho.shape[0]
    rng = np.random.default_rng(190111371 + 2)
    rows = np.sort(rng.choice(n, 48, replace=False))
    t0 = time.perf_counter()
    ax = efie.exact_rows_matvec(rows, x_gpu.astype(np.complex128), rho, w, kappa, chunk=8)
    t = time.perf_counter() - t0
    t_full = t * n / len(rows)
    res = np.linalg.norm(b[rows] - ax) / np.linalg.norm(b[rows])
    log(f"[bench] oracle: {len(rows)} exact rows in {t:.1f}s -> full apply {t_full:.0f}s (extrapolated); "
        f"sampled relres of the GPU solution {res:.2e}")
    return {"value": round(mv_bytes / t_full / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(rows)} seeded rows of the exact matrix-free FP64 product A x at N={n} "
                      f"({t:.1f} s), scaled by N/{len(rows)} to one apply; GB/s = the H-IDBF apply's "
                      f"algorithmic bytes over that time",
            "seconds_per_apply_extrapolated": t_full,
            "gpu_solution_sampled_relres": float(res)}


if __name__ == "__main__":
    main()
