"""Thin Python binding of the hbf C ABI.

``Context`` wraps a device context (hbf_build / hbf_matvec / hbf_precond_apply
/ hbf_solve / hbf_solve_adjoint) and passes torch device tensors and the
current HIP stream through; it only marshals arguments.  ``HostPlan`` wraps the
host-only construction checks (hbf_plan_*), which need no GPU.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi
from ._capi import (HBF_C64, HBF_C128, HBF_PREC_BLOCK_LU, HBF_PREC_NONE, HBF_PREC_PAPER_TRI,  # noqa: F401
                    HbfError, check)

PREC = {"block": HBF_PREC_BLOCK_LU, "paper": HBF_PREC_PAPER_TRI, "none": HBF_PREC_NONE}
DTYPE = {"c64": HBF_C64, "c128": HBF_C128}
METHOD = {"gmres": _capi.HBF_GMRES, "tfqmr": _capi.HBF_TFQMR}


def _curve_struct(curves):
    xy = np.ascontiguousarray(curves.xy, dtype=np.float64)
    off = np.ascontiguousarray(curves.node_off, dtype=np.int64)
    cs = _capi.Curve(len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                     xy.ctypes.data_as(C.POINTER(C.c_double)))
    return cs, (xy, off)


def _opts(dtype="c64", prec="block", z=None, max_nrhs=1, restart=30, device=0, nthreads=0, eta0=0.0,
          cache_plan=0, superleaf=0, verbose=0, host_entries=0):
    keep = []
    zp = None
    if z is not None:
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128)).view(np.float64)
        keep.append(zz)
        zp = zz.ctypes.data_as(C.POINTER(C.c_double))
    o = _capi.BuildOpts(DTYPE[dtype], PREC[prec], eta0, zp, max_nrhs, restart, device, nthreads, cache_plan,
                        superleaf, int(verbose), int(host_entries))
    return o, keep


def hankel2_0(x):
    """The library's own FP64 H0^(2) (host)."""
    lib = _capi.load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty(x.shape, dtype=np.complex128)
    lib.hbf_hankel2_0(x.ctypes.data, x.size, out.ctypes.data)
    return out


class HostPlan:
    """Host-side factorisation evaluated in FP64 on the CPU (construction
    checks; not a compute path of the library)."""

    def __init__(self, curves, kappa, leaf, tol, prec="block", z=None, nthreads=0, lib=None, dtype="c128",
                 superleaf=0, batched_entries=False):
        # batched_entries: evaluate the construction's kernel entries through
        # the batched interface a device build uses (served on the host)
        # dtype: the device storage type whose sweep schedule the plan mirrors
        # (it sets which sweep programs keep their vectors in LDS); the host
        # evaluation is FP64 either way
        self.lib = lib or _capi.load()
        cs, keep = _curve_struct(curves)
        self._keep = list(keep)
        o, k2 = _opts(dtype, prec, z, nthreads=nthreads, superleaf=superleaf, host_entries=2 if batched_entries else 0)
        self._keep += k2
        h = C.c_void_p()
        check(self.lib, self.lib.hbf_plan_build(C.byref(cs), kappa, leaf, tol, C.byref(o), C.byref(h)))
        self.h = h
        st = _capi.Stats()
        check(self.lib, self.lib.hbf_plan_stats(self.h, C.byref(st)))
        self.stats = st.as_dict()
        self.n = int(st.n)

    def _vec_call(self, fn, x, adjoint):
        x = np.ascontiguousarray(np.atleast_2d(np.asarray(x, dtype=np.complex128)))
        y = np.empty_like(x)
        check(self.lib, fn(self.h, x.ctypes.data, y.ctypes.data, x.shape[0], int(adjoint)))
        return y

    def apply(self, x, adjoint=False):
        y = self._vec_call(self.lib.hbf_plan_apply, x, adjoint)
        return y[0] if np.ndim(x) == 1 else y

    def precond(self, r, adjoint=False):
        y = self._vec_call(self.lib.hbf_plan_precond, r, adjoint)
        return y[0] if np.ndim(r) == 1 else y

    def entries(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty((len(rows), len(cols)), dtype=np.complex128)
        check(self.lib, self.lib.hbf_plan_entries(self.h, rows.ctypes.data_as(C.POINTER(C.c_int64)), len(rows),
                                                  cols.ctypes.data_as(C.POINTER(C.c_int64)), len(cols),
                                                  out.ctypes.data))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.hbf_plan_free(self.h)
            self.h = None


def _torch():
    import torch
    return torch


def _stream_ptr(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """Device H-IDBF-LU context.  Vectors are torch tensors on the context's
    device, shape (N,) or (nrhs, N), complex64 or complex128."""

    def __init__(self, curves, kappa, leaf, tol, dtype="c64", prec="block", z=None, max_nrhs=1, restart=30,
                 device=0, nthreads=0, cache_plan=False, superleaf=0, verbose=False, host_entries=False):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("hbf.Context needs a HIP device")
        self.lib = _capi.load()
        self.device = torch.device("cuda", device)
        cs, keep = _curve_struct(curves)
        o, k2 = _opts(dtype, prec, z, max_nrhs=max_nrhs, restart=restart, device=device, nthreads=nthreads,
                      cache_plan=int(cache_plan), superleaf=superleaf, verbose=verbose,
                      host_entries=host_entries)
        h = C.c_void_p()
        check(self.lib, self.lib.hbf_build(C.byref(cs), kappa, leaf, tol, C.byref(o), C.byref(h)))
        del keep, k2
        self.h = h
        self.dtype = dtype
        self.prec = prec
        self.max_nrhs = max_nrhs
        self.n = int(self.lib.hbf_size(self.h))
        st = _capi.Stats()
        check(self.lib, self.lib.hbf_stats(self.h, C.byref(st)))
        self.stats = st.as_dict()

    # -- helpers --------------------------------------------------------------
    def _prep(self, v, io):
        torch = _torch()
        want = torch.complex64 if io == "c64" else torch.complex128
        if v.device != self.device or v.dtype != want:
            raise ValueError(f"expected a {want} tensor on {self.device}, got {v.dtype} on {v.device}")
        v2 = v.reshape(-1, self.n)
        if not v2.is_contiguous():
            v2 = v2.contiguous()
        return v2

    def matvec(self, x, adjoint=False, io=None):
        io = io or ("c64" if x.dtype == _torch().complex64 else "c128")
        xx = self._prep(x, io)
        y = _torch().empty_like(xx)
        check(self.lib, self.lib.hbf_matvec(self.h, C.c_void_p(xx.data_ptr()), C.c_void_p(y.data_ptr()),
                                            xx.shape[0], DTYPE[io], int(adjoint), _stream_ptr(_torch(), self.device)))
        return y.reshape(x.shape)

    def matvec_noalloc(self, x, adjoint=False, io=None):
        """hbf_matvec_noalloc: the same product with the library's fixed
        per-device scratch instead of the context's workspace."""
        io = io or ("c64" if x.dtype == _torch().complex64 else "c128")
        xx = self._prep(x, io)
        y = _torch().empty_like(xx)
        check(self.lib, self.lib.hbf_matvec_noalloc(self.h, C.c_void_p(xx.data_ptr()), C.c_void_p(y.data_ptr()),
                                                    xx.shape[0], DTYPE[io], int(adjoint),
                                                    _stream_ptr(_torch(), self.device)))
        return y.reshape(x.shape)

    def precond(self, r, adjoint=False):
        io = self.dtype
        rr = self._prep(r, io)
        z = _torch().empty_like(rr)
        check(self.lib, self.lib.hbf_precond_apply(self.h, C.c_void_p(rr.data_ptr()), C.c_void_p(z.data_ptr()),
                                                   rr.shape[0], DTYPE[io], int(adjoint),
                                                   _stream_ptr(_torch(), self.device)))
        return z.reshape(r.shape)

    def _solve(self, fn, b, tol, restart, max_iters, max_refine, mixed, x0, inner_tol, method):
        torch = _torch()
        io = "c64" if b.dtype == torch.complex64 else "c128"
        bb = self._prep(b, io)
        if x0 is not None:
            x = self._prep(x0, io).clone()
        else:
            x = torch.empty_like(bb)
        nr = bb.shape[0]
        o = _capi.SolveOpts(tol, restart, max_iters, max_refine, int(mixed), int(x0 is not None), inner_tol,
                            METHOD[method])
        info = (_capi.SolveInfo * nr)()
        st = fn(self.h, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), nr, DTYPE[io], C.byref(o), info,
                _stream_ptr(torch, self.device))
        check(self.lib, st)
        infos = [dict(iters=i.iters, refinements=i.refinements, converged=bool(i.converged), relres=i.relres)
                 for i in info]
        return x.reshape(b.shape), infos, st

    def solve(self, b, tol=1e-6, restart=0, max_iters=0, max_refine=0, mixed=None, x0=None, inner_tol=0.0,
              method="gmres"):
        if mixed is None:
            mixed = self.dtype == "c64"
        return self._solve(self.lib.hbf_solve, b, tol, restart, max_iters, max_refine, mixed, x0, inner_tol, method)

    def solve_adjoint(self, g, tol=1e-6, restart=0, max_iters=0, max_refine=0, mixed=None, x0=None, inner_tol=0.0,
                      method="gmres"):
        if mixed is None:
            mixed = self.dtype == "c64"
        return self._solve(self.lib.hbf_solve_adjoint, g, tol, restart, max_iters, max_refine, mixed, x0, inner_tol,
                           method)

    def impedance_grad(self, lam, x):
        """-sum over right-hand sides of lam * conj(x) (hbf_impedance_grad), shape (N,)."""
        torch = _torch()
        io = "c64" if x.dtype == torch.complex64 else "c128"
        ll = self._prep(lam, io)
        xx = self._prep(x, io)
        if ll.shape != xx.shape:
            raise ValueError("lam and x must have the same shape")
        g = torch.empty(self.n, dtype=xx.dtype, device=self.device)
        check(self.lib, self.lib.hbf_impedance_grad(self.h, C.c_void_p(ll.data_ptr()), C.c_void_p(xx.data_ptr()),
                                                    xx.shape[0], DTYPE[io], C.c_void_p(g.data_ptr()),
                                                    _stream_ptr(torch, self.device)))
        return g

    def tune(self, key, value):
        check(self.lib, self.lib.hbf_tune(self.h, key.encode(), int(value)))

    def set_impedance(self, z):
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128)).view(np.float64)
        if zz.size != 2 * self.n:
            raise ValueError(f"impedance needs {self.n} values, got {zz.size // 2}")
        check(self.lib, self.lib.hbf_set_impedance(self.h, zz.ctypes.data_as(C.POINTER(C.c_double))))
        st = _capi.Stats()
        check(self.lib, self.lib.hbf_stats(self.h, C.byref(st)))
        self.stats = st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.lib.hbf_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
