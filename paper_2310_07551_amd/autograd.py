"""Differentiable split-ETD3 integration (torch.autograd.Function).

The forward pass runs the library's time stepping and keeps the state every
`checkpoint` steps; the backward pass recomputes each segment's states from
its checkpoint and runs the library's adjoint step (setd_etd_adjoint_step)
backwards through them.  Gradients: with respect to the initial state, the
reaction parameters and the diffusion coefficient of each component, where
the matrices are A_mu^(c) = diff[c] * D_mu^(c).

Argument marshalling only: every step, forward and adjoint, runs in libsetd.
"""
from __future__ import annotations

from typing import Sequence

from . import Context, PREC_F64


def _torch():
    import torch
    return torch


class _Integrate(_torch().autograd.Function):
    @staticmethod
    def forward(fctx, u0, params, diff, spec):
        torch = _torch()
        dims, D, g_kind, tau, nsteps, checkpoint, diff_components = spec[:7]
        ncomp = len(D)
        dvals = [float(x) for x in diff.detach().cpu()]
        pvals = [float(x) for x in params.detach().cpu()]
        A = [[(dvals[c] * Dm).contiguous() for Dm in D[c]] for c in range(ncomp)]
        ctx = Context(dims, A, tau, prec=PREC_F64)
        u = u0.detach().clone().contiguous()
        checkpoints = [u.clone()]
        done = 0
        while done < nsteps:
            k = min(checkpoint, nsteps - done)
            ctx.step(u, k, g_kind, pvals)
            done += k
            if done < nsteps:
                checkpoints.append(u.clone())
        fctx.setd = (ctx, checkpoints, pvals, dvals, spec)
        fctx.devices = (params.device, diff.device)
        return u

    @staticmethod
    def backward(fctx, grad_u):
        torch = _torch()
        ctx, checkpoints, pvals, dvals, spec = fctx.setd
        dims, D, g_kind, tau, nsteps, checkpoint, diff_components = spec[:7]
        ncomp = len(D)
        ubar = grad_u.detach().to(torch.float64).contiguous().clone()
        grad = torch.zeros(len(pvals) + ncomp, dtype=torch.float64, device=ubar.device)
        work = torch.empty_like(ubar)
        # diffusion-size gradients only for the components asked for (each
        # costs 2d extra Tucker groups per step)
        mask = 0
        if fctx.needs_input_grad[2]:
            for c in (range(ncomp) if diff_components is None else diff_components):
                mask |= 1 << int(c)
        record = spec_record(spec)
        recs = None
        for seg in range(len(checkpoints) - 1, -1, -1):
            k = min(checkpoint, nsteps - seg * checkpoint)
            states = torch.empty((k, ubar.numel()), dtype=torch.float64, device=ubar.device)
            if record and recs is None:
                # stage quantities of every step of a segment (6 ncomp N each)
                recs = torch.empty((checkpoint, 6 * ubar.numel()), dtype=torch.float64, device=ubar.device)
            work.copy_(checkpoints[seg])
            for j in range(k):
                states[j].copy_(work)
                if record:
                    ctx.step_record(work, recs[j], g_kind, pvals)
                elif j + 1 < k:
                    ctx.step(work, 1, g_kind, pvals)
            for j in range(k - 1, -1, -1):
                ctx.adjoint_step(states[j], ubar, g_kind, pvals, grad, sigma_mask=mask,
                                 rec=recs[j] if record else None)
        g = grad.cpu()
        gp = g[:len(pvals)].clone()
        gd = torch.tensor([g[len(pvals) + c].item() / dvals[c] if (mask >> c) & 1 else 0.0 for c in range(ncomp)],
                          dtype=torch.float64)
        fctx.setd = None
        ctx.close()
        return ubar, gp.to(fctx.devices[0]), gd.to(fctx.devices[1]), None


def spec_record(spec) -> bool:
    return bool(spec[7]) if len(spec) > 7 else True


def integrate(u0, params, diff, *, dims: Sequence[int], D, g_kind: int, tau: float, nsteps: int,
              checkpoint: int = 20, diff_components=None, record: bool = True):
    """u(T) after nsteps split-ETD3 steps from u0 (flat FP64 device tensor,
    component-major), differentiable in u0, params (1-D tensor of reaction
    parameters) and diff (1-D tensor, one diffusion coefficient per
    component; A_mu^(c) = diff[c] * D[c][mu], D column-major FP64 device
    matrices).  diff_components: the components whose diffusion gradient is
    wanted (default all; the others get 0).  The backward pass steps forward
    from each checkpoint again; with record (default) those steps keep their
    stage quantities (6 ncomp N doubles per step of a segment) so that the
    adjoint steps need not recompute them."""
    if checkpoint < 1:
        raise ValueError("checkpoint must be >= 1")
    comps = None if diff_components is None else tuple(int(c) for c in diff_components)
    spec = (tuple(int(x) for x in dims), D, int(g_kind), float(tau), int(nsteps), int(checkpoint), comps,
            bool(record))
    return _Integrate.apply(u0, params, diff, spec)
