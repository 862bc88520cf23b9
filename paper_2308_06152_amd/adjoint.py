"""Misfit and adjoint-state gradient with respect to s = 1/c^2 for a set of
sources at one frequency, as a torch.autograd.Function.

For k = omega sqrt(s) (the model problem of Section 2), the forward pass
solves A(s) u_q = b_q for all sources q in one batched solve and returns
J = 1/2 sum_q ||R u_q - d_q||^2; the backward pass solves the adjoint systems
A^H lambda_q = R^T (R u_q - d_q) (batched, by the complex-symmetric scaling
of A) and accumulates g = -Re(conj(lambda_q) dA/ds u_q).  Every step runs in
libhelmdefl.so; this module only holds the tensors between the calls.  The
forward wavefields are kept for the backward pass (at nrhs x ny x nx x 16
bytes; recompute them, or split the sources into groups, when that exceeds
the device memory).
"""
from __future__ import annotations

import math

import torch

from . import helmdefl as H


class HelmholtzMisfit(torch.autograd.Function):
    """J(s) = 1/2 sum_q ||R u_q(s) - d_q||^2.

    apply(s, omega, grid, sources, rec, d_obs, opts) with s a CUDA float64
    (ny, nx) tensor, grid = (nx, ny, hx, hy, bc), sources (nrhs, ny, nx)
    complex128, rec int32 node indices, d_obs (nrhs, nrec) complex128, opts a
    dict of solver options.  Returns J (0-dim float64)."""

    @staticmethod
    def forward(ctx, s, omega, grid, sources, rec, d_obs, opts):
        nx, ny, hx, hy, bc = grid
        k = (omega * torch.sqrt(s)).contiguous()
        S = H.Solver(nx, ny, hx, hy, bc, k=k, **opts)
        u, info = S.solve(sources)
        if not all(i["converged"] for i in info):
            raise H.HelmError(H.HELM_ENOCONV, "forward solve")
        _, f, J = S.receivers(rec, u, d_obs)
        ctx.S, ctx.omega = S, omega
        ctx.save_for_backward(u, f)
        ctx.forward_info = info
        return J.sum()

    @staticmethod
    def backward(ctx, gJ):
        u, f = ctx.saved_tensors
        lam, info = ctx.S.adjoint_solve(f)
        if not all(i["converged"] for i in info):
            raise H.HelmError(H.HELM_ENOCONV, "adjoint solve")
        g = ctx.S.gradient_s(ctx.omega, u, lam)
        ctx.S.close()
        return g * gJ, None, None, None, None, None, None


def misfit(s, omega, grid, sources, rec, d_obs, **opts):
    """J(s) with autograd support (see HelmholtzMisfit)."""
    return HelmholtzMisfit.apply(s, omega, grid, sources, rec, d_obs, opts)


def angular(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz
