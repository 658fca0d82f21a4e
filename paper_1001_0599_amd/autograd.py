"""P, P^T and the smoothed TV sum as torch.autograd.Functions over libcbct.

The backward of the projector is the hand-written adjoint gather (its exact transpose), and
the backward of the adjoint is the projector; the TV sum S(f) = sum sqrt(|D f|^2 + eps^2)
(boundary conditions of the paper's Section II.B) takes its gradient from the TV kernel.
Inputs may carry a leading batch axis; each volume of the batch is projected on the current
stream in turn.
"""
from __future__ import annotations

import torch


def _vol_batch(x: torch.Tensor, shape):
    if tuple(x.shape) == tuple(shape):
        return x.unsqueeze(0), False
    if x.dim() == len(shape) + 1 and tuple(x.shape[1:]) == tuple(shape):
        return x, True
    raise ValueError("expected shape %s or (B, *%s), got %s" % (tuple(shape), tuple(shape), tuple(x.shape)))


def _project(plan, f: torch.Tensor, level: int) -> torch.Tensor:
    fb, batched = _vol_batch(f, plan.vol_shape(level))
    fb = fb.contiguous()
    out = torch.empty((fb.shape[0],) + tuple(plan.proj_shape(level)), dtype=torch.float32, device=f.device)
    ws = torch.empty(plan.forward_workspace_bytes(level), dtype=torch.uint8, device=f.device)
    for b in range(fb.shape[0]):
        plan.forward(fb[b], level=level, out=out[b], workspace=ws)
    return out if batched else out[0]


def _backproject(plan, y: torch.Tensor, level: int) -> torch.Tensor:
    yb, batched = _vol_batch(y, plan.proj_shape(level))
    yb = yb.contiguous()
    out = torch.empty((yb.shape[0],) + tuple(plan.vol_shape(level)), dtype=torch.float32, device=y.device)
    ws = torch.empty(plan.adjoint_workspace_bytes(level), dtype=torch.uint8, device=y.device)
    for b in range(yb.shape[0]):
        plan.adjoint(yb[b], level=level, out=out[b], workspace=ws)
    return out if batched else out[0]


class ForwardProject(torch.autograd.Function):
    """y = P f; dL/df = P^T dL/dy."""

    @staticmethod
    def forward(ctx, f, plan, level=0):
        ctx.plan, ctx.level = plan, level
        return _project(plan, f.detach(), level)

    @staticmethod
    def backward(ctx, grad_y):
        return _backproject(ctx.plan, grad_y.contiguous(), ctx.level), None, None


class BackProject(torch.autograd.Function):
    """f = P^T y; dL/dy = P dL/df."""

    @staticmethod
    def forward(ctx, y, plan, level=0):
        ctx.plan, ctx.level = plan, level
        return _backproject(plan, y.detach(), level)

    @staticmethod
    def backward(ctx, grad_f):
        return _project(ctx.plan, grad_f.contiguous(), ctx.level), None, None


class TVSum(torch.autograd.Function):
    """S(f) = sum_voxels sqrt(|D f|^2 + eps^2) (summed over the batch); dS/df from the TV kernel."""

    @staticmethod
    def forward(ctx, f, plan, eps=1e-5, level=0):
        fb, batched = _vol_batch(f.detach(), plan.vol_shape(level))
        fb = fb.contiguous()
        grads = torch.empty_like(fb)
        total = 0.0
        for b in range(fb.shape[0]):
            s, _ = plan.tv_energy_grad(fb[b], eps, level=level, grad=grads[b])
            total += s
        ctx.save_for_backward(grads if batched else grads[0])
        return torch.tensor(total, dtype=torch.float64, device=f.device)

    @staticmethod
    def backward(ctx, grad_s):
        (g,) = ctx.saved_tensors
        return g * grad_s.to(g.dtype), None, None, None


def project(f, plan, level: int = 0):
    return ForwardProject.apply(f, plan, level)


def backproject(y, plan, level: int = 0):
    return BackProject.apply(y, plan, level)


def tv_sum(f, plan, eps: float = 1e-5, level: int = 0):
    return TVSum.apply(f, plan, eps, level)
