"""torch.autograd.Function around libvrk: the forward pass is the Kaczmarz
solve, the backward pass the library's adjoint solve (implicit
differentiation: the same sweep on the same system with right-hand side
H g; no iterates are stored).

Gradients follow torch's complex convention (grad = 2 dL/d conj(z)); the
gradient with respect to H is nonzero only on the VR band entries, the
only entries of H the precoder depends on (under the subarray VR model, only
on the visible subarrays).
"""
from __future__ import annotations

import numpy as np
import torch

from . import vrk


class KaczmarzRZF(torch.autograd.Function):
    """x_b = H^H (H H^H + xi I)^-1 s_b for every row s_b of S."""

    @staticmethod
    def forward(ctx, H, S, xi, vr_start, vr_len, opts, vr_mask=None, n_sub=0):
        if not H.is_cuda or not S.is_cuda:
            raise ValueError("KaczmarzRZF needs device tensors")
        if H.dtype not in (torch.complex64, torch.complex128) or S.dtype != H.dtype:
            raise ValueError("H and S must share one complex dtype (got %s and %s)" % (H.dtype, S.dtype))
        dtype = "c128" if H.dtype == torch.complex128 else "c64"
        xi_val = float(xi) if not torch.is_tensor(xi) else float(xi.detach().cpu())
        Hc = H.detach().contiguous()
        Sc = S.detach().reshape(-1, H.shape[0]).contiguous()
        B = Sc.shape[0]
        X = torch.empty((B, H.shape[1]), dtype=H.dtype, device=H.device)
        V = torch.empty((B, H.shape[0]), dtype=H.dtype, device=H.device)
        GX = torch.zeros_like(X)
        GH = torch.zeros_like(Hc)
        GS = torch.zeros_like(Sc)
        gxi = torch.zeros(1, dtype=torch.float64, device=H.device)
        o = vrk.options(dtype=dtype, **(opts or {}))
        plan = vrk.Plan([vrk.ProblemSpec(Hc, vr_start, vr_len, xi_val, Sc, X, V, GX, GH, GS, gxi,
                                         vr_mask, n_sub)], o)
        stats = plan.stats_buffers()
        plan.solve(stats=stats)
        ctx.plan = plan
        ctx.bufs = (GX, GH, GS, gxi)
        ctx.stats = stats
        ctx.xi_is_tensor = torch.is_tensor(xi)
        ctx.s_shape = S.shape
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors   # raises if X was modified in place
        GX, GH, GS, gxi = ctx.bufs
        GX.copy_(gX.reshape(GX.shape))
        GH.zero_()
        ctx.plan.solve_adjoint()
        gH = GH.clone()
        gS = GS.clone().reshape(ctx.s_shape)
        gx = gxi[0].clone() if ctx.xi_is_tensor else None
        return gH, gS, gx, None, None, None, None, None


def rzf_precode(H, S, xi, vr_start, vr_len, vr_mask=None, n_sub=0, **opts):
    """Differentiable precoding of the rows of S (B x K) for channel H
    (K x Nt) with per-user VR [vr_start, vr_start + vr_len) (the hulls of
    the visible subarrays when vr_mask / n_sub give the subarray model).
    Options as vrk.options (variant, tol, engine, ...)."""
    vs = np.ascontiguousarray(vr_start, dtype=np.int32)
    vl = np.ascontiguousarray(vr_len, dtype=np.int32)
    vm = None if vr_mask is None else np.ascontiguousarray(vr_mask, dtype=np.uint64)
    return KaczmarzRZF.apply(H, S, xi, vs, vl, opts, vm, int(n_sub))
