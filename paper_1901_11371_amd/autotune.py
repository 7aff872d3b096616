"""Autotuner for the execution parameters of an hbf context.

It times the applications one GMRES iteration makes (one preconditioner
application and one matvec) for a given number of right-hand sides over the
candidate values of the parameters exposed by ``hbf_tune`` and keeps the
fastest:

* ``prog_levels``: subtrees of at most 2^p leaves are swept inside one
  workgroup program (deep subtrees: fewer launches and cheap step
  barriers, but one workgroup per RHS chunk streams their factors);
* the stage kernel of the matvec and, separately, of the big sweep blocks
  (with complex64 factors and 8 or more RHS also the matrix-core kernel at
  16, 32 or 64 RHS per wave):
  the software-pipelined wave teams (``pipe_max_r`` / ``sweep_pipe_max_r``
  >= nrhs), or one unit per wave / workgroup (``wave_units``); and whether
  the sweeps' stage launches use the pipelined kernel with one RHS per chunk
  (``sweep_rc1``).

Results are cached in a JSON table keyed by (N, nrhs, dtype, preconditioner)
so later runs of the same shape apply them without timing.
"""
from __future__ import annotations

import json
import os

import torch

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "autotune.json")

# stage-kernel variants: name -> hbf_tune settings
_VALU = {"mfma": 0, "mfma_min_r": 8, "mfma_tiles": 4, "sweep_mfma_tiles": 1}
_NO_PIPE = {"pipe_max_r": 4, "sweep_pipe_max_r": 4, "wave_units": 1, "sweep_rc1": 0}
KERNELS = {
    "pipe": lambda R: {"pipe_max_r": max(R, 1), "sweep_pipe_max_r": max(R, 1), "wave_units": 1, "sweep_rc1": 0,
                       **_VALU},
    "wave": lambda R: {"pipe_max_r": 0, "sweep_pipe_max_r": 0, "wave_units": 1, "sweep_rc1": 0, **_VALU},
    "wave+sweep_pipe": lambda R: {"pipe_max_r": 0, "sweep_pipe_max_r": max(R, 1), "wave_units": 1, "sweep_rc1": 0,
                                  **_VALU},
    "pipe+sweep_wave": lambda R: {"pipe_max_r": max(R, 1), "sweep_pipe_max_r": 0, "wave_units": 1, "sweep_rc1": 0,
                                  **_VALU},
    "wave+rc1": lambda R: {"pipe_max_r": 0, "sweep_pipe_max_r": 0, "wave_units": 1, "sweep_rc1": 1, **_VALU},
    # matrix-core stage launches (complex64 only): the matvec at 64 right-hand
    # sides per wave, the sweeps' launches at 16, 32 or 64
    "mfma16": lambda R: {**_NO_PIPE, "mfma": 1, "mfma_min_r": 1, "mfma_tiles": 4, "sweep_mfma_tiles": 1},
    "mfma32": lambda R: {**_NO_PIPE, "mfma": 1, "mfma_min_r": 1, "mfma_tiles": 4, "sweep_mfma_tiles": 2},
    "mfma64": lambda R: {**_NO_PIPE, "mfma": 1, "mfma_min_r": 1, "mfma_tiles": 4, "sweep_mfma_tiles": 4},
}


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


def autotune(ctx, nrhs=1, reps=2, prog_levels=(4, 5, 6, 7, 8), kernels=tuple(KERNELS), path=DEFAULT_TABLE,
             verbose=False):
    """Time the candidates on `ctx` (an hbf.Context) and keep the best."""
    dt = torch.complex64 if ctx.dtype == "c64" else torch.complex128
    shape = (nrhs, ctx.n) if nrhs > 1 else (ctx.n,)
    x = torch.randn(shape, dtype=dt, device=ctx.device)
    best = {}
    timings = {}

    def say(msg):
        if verbose:
            print(f"[autotune] {msg}", flush=True)

    if ctx.prec != "none":
        res = {}
        for p in prog_levels:
            ctx.tune("prog_levels", p)
            res[p] = _time(lambda: ctx.precond(x), reps)
            say(f"prog_levels={p}: precond {res[p]:.3f} ms")
        p = min(res, key=res.get)
        best["prog_levels"] = p
        timings["precond_ms"] = res
        ctx.tune("prog_levels", p)
    res = {}
    for name in kernels:
        if name.startswith("mfma") and (ctx.dtype != "c64" or nrhs < 8):
            continue
        for k, v in KERNELS[name](nrhs).items():
            ctx.tune(k, v)
        t = _time(lambda: ctx.matvec(x), reps)
        if ctx.prec != "none":
            t += _time(lambda: ctx.precond(x), reps)
        res[name] = t
        say(f"kernel={name}: matvec + precond {t:.3f} ms")
    name = min(res, key=res.get)
    settings = KERNELS[name](nrhs)
    for k, v in settings.items():
        ctx.tune(k, v)
    best.update(settings)
    timings["iteration_ms"] = res
    table = load_table(path)
    table[_key(ctx, nrhs)] = {"params": best, "kernel": name,
                              "timings_ms": {k: {str(a): b for a, b in v.items()} for k, v in timings.items()}}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return best
