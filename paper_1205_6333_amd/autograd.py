"""torch.autograd wrappers of the product and of the Euler time loop.

The forward and backward passes are library calls: mobility_apply /
mobility_adjoint for one product, sd_run / sd_run_adjoint (checkpointed
recomputation) for the time loop.  Positions and forces enter as (n, 3)
float64 CUDA tensors and are staged into the record layout by sd_pack.
"""
from __future__ import annotations

import torch

from . import binding as B


class MobilityFn(torch.autograd.Function):
    """v = M(x) F with gradients d/dx [g . v] and M(x) g (= M(x)^T g)."""

    @staticmethod
    def forward(ctx, x, F, params, precision):
        pos = B.sd_pack(x.contiguous(), precision)
        frc = B.sd_pack(F.contiguous(), precision)
        v = B.mobility_apply(pos, frc, params=params, precision=precision)
        ctx.save_for_backward(pos, frc)
        ctx.params, ctx.precision = params, precision
        return v

    @staticmethod
    def backward(ctx, g):
        pos, frc = ctx.saved_tensors
        lam = B.sd_pack(g.contiguous(), ctx.precision)
        gx, gF = B.mobility_adjoint(pos, frc, lam, params=ctx.params, precision=ctx.precision,
                                    want_force=ctx.needs_input_grad[1])
        return gx if ctx.needs_input_grad[0] else None, gF, None, None


def mobility(x, F, params=None, precision: int = B.SD_FP32_KAHAN):
    """Differentiable mobility product for (n, 3) float64 CUDA tensors."""
    return MobilityFn.apply(x, F, params if params is not None else B.params(), int(precision))


class SdRunFn(torch.autograd.Function):
    """x_steps of `steps` explicit Euler steps from x0 under constant forces F;
    the backward pass recomputes every segment of `checkpoint_every` steps from
    the checkpoints written by the forward pass."""

    @staticmethod
    def forward(ctx, x0, F, dt, steps, checkpoint_every, params, precision):
        n = x0.shape[0]
        x = x0.detach().clone().contiguous()
        frc = B.sd_pack(F.contiguous(), precision)
        ck = torch.empty((steps // checkpoint_every + 1) * n * 3, dtype=torch.float64,
                         device=x0.device)
        B.sd_run(x, frc, dt, steps, checkpoints=ck, checkpoint_every=checkpoint_every,
                 params=params, precision=precision)
        ctx.save_for_backward(x0.detach().contiguous(), frc, ck)
        ctx.cfg = (dt, steps, checkpoint_every, params, precision)
        return x

    @staticmethod
    def backward(ctx, gxN):
        x0, frc, ck = ctx.saved_tensors
        dt, steps, every, params, precision = ctx.cfg
        gx0, gF = B.sd_run_adjoint(x0, frc, dt, steps, gxN.contiguous(), checkpoints=ck,
                                   checkpoint_every=every, params=params, precision=precision)
        return gx0, gF, None, None, None, None, None


def run(x0, F, dt: float, steps: int, checkpoint_every: int = 20, params=None,
        precision: int = B.SD_FP32_KAHAN):
    """Differentiable explicit-Euler trajectory end point x_steps."""
    return SdRunFn.apply(x0, F, float(dt), int(steps), int(checkpoint_every),
                         params if params is not None else B.params(), int(precision))
