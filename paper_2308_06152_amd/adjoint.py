"""Misfit and adjoint-state gradient with respect to s = 1/c^2 for a set of
sources at one frequency, as a torch.autograd.Function.

For k = omega sqrt(s) (the model problem of Section 2), the forward pass
solves A(s) u_q = b_q for all sources q in batched solves and returns
J = 1/2 sum_q ||R u_q - d_q||^2; the backward pass solves the adjoint systems
A^H lambda_q = R^T (R u_q - d_q) (batched, by the complex-symmetric scaling
of A) and accumulates g = -Re(conj(lambda_q) dA/ds u_q).  Every step runs in
libhelmdefl.so; this module only holds the tensors between the calls.

Memory: the forward wavefields take nshot x ny x nx x 16 bytes.  With
`max_field_bytes` set and the wavefields larger than that, they are not kept:
the backward pass solves the forward problems again, `shot_group` sources at a
time (each group's wavefields are recomputed, used for its adjoint solve and
gradient, and dropped), so the peak holds one group's fields.
"""
from __future__ import annotations

import math

import torch

from . import helmdefl as H


def _solve(S, b, what):
    u, info = S.solve(b)
    if not all(i["converged"] for i in info):
        raise H.HelmError(H.HELM_ENOCONV, what)
    return u


class HelmholtzMisfit(torch.autograd.Function):
    """J(s) = 1/2 sum_q ||R u_q(s) - d_q||^2.

    apply(s, omega, grid, sources, rec, d_obs, opts, max_field_bytes,
    shot_group) with s a CUDA float64 (ny, nx) tensor, grid = (nx, ny, hx, hy,
    bc), sources (nrhs, ny, nx) complex128, rec int32 node indices, d_obs
    (nrhs, nrec) complex128, opts a dict of solver options.  Returns J (0-dim
    float64)."""

    @staticmethod
    def forward(ctx, s, omega, grid, sources, rec, d_obs, opts, max_field_bytes, shot_group):
        nx, ny, hx, hy, bc = grid
        k = (omega * torch.sqrt(s)).contiguous()
        S = H.Solver(nx, ny, hx, hy, bc, k=k, **opts)
        nshot = sources.shape[0]
        field_bytes = nshot * ny * nx * 16
        recompute = max_field_bytes is not None and field_bytes > max_field_bytes
        group = nshot if not recompute else max(1, min(shot_group or nshot, nshot))
        J = torch.zeros((), dtype=torch.float64, device=s.device)
        us, fs = [], []
        for q0 in range(0, nshot, group):
            u = _solve(S, sources[q0:q0 + group].contiguous(), "forward solve")
            _, f, Jq = S.receivers(rec, u, d_obs[q0:q0 + group].contiguous())
            J = J + Jq.sum()
            if not recompute:
                us.append(u)
                fs.append(f)
        ctx.S, ctx.omega, ctx.group, ctx.recompute = S, omega, group, recompute
        if recompute:
            ctx.save_for_backward(sources, rec, d_obs)
        else:
            ctx.save_for_backward(torch.cat(us), torch.cat(fs))
        return J

    @staticmethod
    def backward(ctx, gJ):
        S = ctx.S
        if ctx.recompute:
            sources, rec, d_obs = ctx.saved_tensors
            g = None
            for q0 in range(0, sources.shape[0], ctx.group):
                u = _solve(S, sources[q0:q0 + ctx.group].contiguous(), "forward recompute")
                _, f, _ = S.receivers(rec, u, d_obs[q0:q0 + ctx.group].contiguous())
                lam, info = S.adjoint_solve(f)
                if not all(i["converged"] for i in info):
                    raise H.HelmError(H.HELM_ENOCONV, "adjoint solve")
                g = S.gradient_s(ctx.omega, u, lam, g)
                del u, f, lam
        else:
            u, f = ctx.saved_tensors
            lam, info = S.adjoint_solve(f)
            if not all(i["converged"] for i in info):
                raise H.HelmError(H.HELM_ENOCONV, "adjoint solve")
            g = S.gradient_s(ctx.omega, u, lam)
        S.close()
        return g * gJ, None, None, None, None, None, None, None, None


def misfit(s, omega, grid, sources, rec, d_obs, max_field_bytes=None, shot_group=None, **opts):
    """J(s) with autograd support (see HelmholtzMisfit).  max_field_bytes:
    recompute the forward wavefields in the backward pass, shot_group sources
    at a time, when keeping all of them would take more than this."""
    return HelmholtzMisfit.apply(s, omega, grid, sources, rec, d_obs, opts, max_field_bytes,
                                 shot_group)


def angular(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz
