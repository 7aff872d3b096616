"""Autotuner for the execution parameters of an hbf context.

It times the preconditioner application (the latency-bound sweeps) and the
matvec for a given number of right-hand sides over the candidate values of
each parameter exposed by ``hbf_tune`` and keeps the fastest:

* ``prog_levels``: subtrees of at most 2^p leaves are swept inside one
  workgroup program (deep subtrees: fewer launches, but a single workgroup
  per RHS chunk streams their factors);
* ``r1_max_blocks``: persistent grid size of the one-RHS stage kernel.

Results are cached in a JSON table keyed by (N, nrhs, dtype, preconditioner)
so later runs of the same shape apply them without timing.
"""
from __future__ import annotations

import json
import os

import torch

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "autotune.json")


def _key(ctx, nrhs):
    return f"N={ctx.n},nrhs={nrhs},dtype={ctx.dtype},prec={ctx.prec}"


def _time(fn, reps):
    dev = torch.device("cuda", 0)
    s = torch.cuda.current_stream(dev)
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def load_table(path=DEFAULT_TABLE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(ctx, nrhs, path=DEFAULT_TABLE):
    """Apply a cached result for this shape; returns it (or None)."""
    entry = load_table(path).get(_key(ctx, nrhs))
    if entry:
        for k, v in entry["params"].items():
            ctx.tune(k, v)
    return entry


def autotune(ctx, nrhs=1, reps=3, prog_levels=(3, 4, 5, 6, 7, 8), r1_blocks=(512, 1024, 2048, 4096),
             path=DEFAULT_TABLE, verbose=False):
    """Time the candidates on `ctx` (an hbf.Context) and keep the best."""
    dt = torch.complex64 if ctx.dtype == "c64" else torch.complex128
    x = torch.randn((nrhs, ctx.n), dtype=dt, device=ctx.device) if nrhs > 1 else \
        torch.randn((ctx.n,), dtype=dt, device=ctx.device)
    best = {}
    timings = {}
    if ctx.prec != "none":
        res = {}
        for p in prog_levels:
            ctx.tune("prog_levels", p)
            res[p] = _time(lambda: ctx.precond(x), reps)
            if verbose:
                print(f"[autotune] prog_levels={p}: precond {res[p]:.3f} ms", flush=True)
        p = min(res, key=res.get)
        best["prog_levels"] = p
        timings["precond_ms"] = res
        ctx.tune("prog_levels", p)
    if nrhs == 1:
        res = {}
        for b in r1_blocks:
            ctx.tune("r1_max_blocks", b)
            res[b] = _time(lambda: ctx.matvec(x), reps * 3)
            if verbose:
                print(f"[autotune] r1_max_blocks={b}: matvec {res[b]:.3f} ms", flush=True)
        b = min(res, key=res.get)
        best["r1_max_blocks"] = b
        timings["matvec_ms"] = res
        ctx.tune("r1_max_blocks", b)
    table = load_table(path)
    table[_key(ctx, nrhs)] = {"params": best, "timings_ms": {k: {str(a): b for a, b in v.items()}
                                                             for k, v in timings.items()}}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return best
