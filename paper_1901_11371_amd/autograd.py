"""Differentiable solve x = (Z + diag(z))^{-1} b through the hbf C ABI.

Forward: hbf_solve (right-preconditioned GMRES with the approximate-LU
preconditioner).  Backward: one adjoint solve lam = A^{-H} g with the
conjugate-transposed butterfly traversal and the preconditioner P^{-H}
(hbf_solve_adjoint); grad_b = lam, and grad_z = -sum over right-hand sides of
lam * conj(x) (A depends on z only through its diagonal), formed on the device
by hbf_impedance_grad.  Gradients follow PyTorch's convention for real losses
of complex tensors (dL/dRe + i dL/dIm).

A solve that misses its tolerance raises (its x, or its gradient, would belong
to an unconverged iterate).  The backward pass re-installs the impedance the
forward pass solved with when the context has been given another one since.
"""
from __future__ import annotations

import numpy as np
import torch

from ._capi import HBF_NOCONV


class SolveNotConverged(RuntimeError):
    """A forward or adjoint solve stopped before reaching its tolerance."""


def _require_converged(status, infos, what):
    if status == HBF_NOCONV or not all(i["converged"] for i in infos):
        worst = max(i["relres"] for i in infos)
        raise SolveNotConverged(f"{what} did not converge (largest relres {worst:.3e}); raise max_iters or "
                                f"loosen tol")


def _install_impedance(hctx, zz):
    if getattr(hctx, "_z_cache", None) is None or not np.array_equal(hctx._z_cache, zz):
        hctx.set_impedance(zz)
        hctx._z_cache = zz.copy()


class _HbfSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, z, hctx, solve_kw):
        zz = None
        if z is not None:
            zz = z.detach().to("cpu", torch.complex128).numpy().copy()
            _install_impedance(hctx, zz)
        x, infos, st = hctx.solve(b.detach(), **solve_kw)
        hctx.last_info = infos
        _require_converged(st, infos, "forward solve")
        ctx.hctx = hctx
        ctx.solve_kw = solve_kw
        ctx.has_z = z is not None
        ctx.z_host = zz
        ctx.save_for_backward(x)
        ctx.z_dtype = z.dtype if z is not None else None
        ctx.z_device = z.device if z is not None else None
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        hctx = ctx.hctx
        if ctx.z_host is not None:
            _install_impedance(hctx, ctx.z_host)
        lam, infos, st = hctx.solve_adjoint(grad_x.contiguous().to(x.dtype), **ctx.solve_kw)
        hctx.last_adjoint_info = infos
        _require_converged(st, infos, "adjoint solve")
        grad_b = lam
        grad_z = None
        if ctx.has_z and ctx.needs_input_grad[1]:
            grad_z = hctx.impedance_grad(lam, x).to(device=ctx.z_device, dtype=ctx.z_dtype)
        return grad_b, grad_z, None, None


def hbf_solve(b: torch.Tensor, hctx, z: torch.Tensor | None = None, **solve_kw) -> torch.Tensor:
    """x = (Z + diag(z))^{-1} b for the context `hctx` (hbf.Context); b is a
    device tensor of shape (N,) or (nrhs, N).  If z is given it replaces the
    context's impedance (leaf blocks are refactored when it changes)."""
    return _HbfSolve.apply(b, z, hctx, solve_kw)


def farfield_objective(x: torch.Tensor, rho: torch.Tensor, w: torch.Tensor, kappa: float,
                       angles: torch.Tensor) -> torch.Tensor:
    """J = sum_m |F(phi_m)|^2 with F(phi) = sum_j w_j x_j exp(+i kappa rho_j . u(phi))
    (a far-field pattern of the induced current; constant prefactor dropped)."""
    ph = kappa * (torch.outer(torch.cos(angles), rho[:, 0]) + torch.outer(torch.sin(angles), rho[:, 1]))
    C = w[None, :] * torch.exp(1j * ph)
    F = C.to(x.dtype) @ x.reshape(-1)
    return (F.abs() ** 2).sum()
