"""Differentiable n-step propagation (torch.autograd), backed by the
library's hand-written adjoint kernels and its checkpoint schedule.

``propagate(fields, coeffs, n, dt)`` returns the six fields after n steps;
gradients flow to the initial fields and to the 12 coefficients (a float64
tensor).  The forward pass keeps the state every ``seg`` steps (default
ceil(sqrt(2 n)), a workspace of O(sqrt(n)) fields) and the E fields of the
last two segments; the backward pass recomputes each earlier segment from its
checkpoint (the previous segment on a second stream while it reverses the
current one) and runs the adjoint steps in reverse (see include/xfdtd.h).
"""
from __future__ import annotations

import torch

from .solver import Solver


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, n, dt, spacing, seg, allow_unstable, *fields):
        out = [f.detach().contiguous().clone() for f in fields]
        c = [float(v) for v in coeffs.detach().cpu().tolist()]
        solver = Solver(out, dt, c, spacing=spacing, scratch=False, allow_unstable=allow_unstable)
        nbytes = solver.grad_workspace_bytes(n, seg)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=out[0].device)
        solver.grad_forward(n, ws, seg)
        ctx.solver, ctx.ws, ctx.n, ctx.seg = solver, ws, n, seg
        ctx.coeff_device = coeffs.device
        return tuple(out)

    @staticmethod
    def backward(ctx, *grads):
        if ctx.ws is None:
            raise RuntimeError("propagate: the backward pass consumes the forward pass's checkpoints; "
                               "run propagate again for a second backward pass")
        solver = ctx.solver
        ref = solver.fields[0]
        lam = [torch.zeros_like(ref) if g is None else g.detach().to(ref.dtype).contiguous().clone()
               for g in grads]
        gc = solver.grad_backward(ctx.n, ctx.ws, lam, ctx.seg)
        ctx.ws = None
        gcoef = torch.tensor(gc, dtype=torch.float64, device=ctx.coeff_device)
        return (gcoef, None, None, None, None, None, *lam)


def propagate(fields, coeffs, n, dt, spacing=(1.0, 1.0, 1.0), seg=0, allow_unstable=False):
    """Six fields after n steps, differentiable w.r.t. ``fields`` and ``coeffs``.

    fields: six CUDA tensors (nz, ny, nx), float32 or float64.
    coeffs: float64 tensor of 12 coefficients (order of include/xfdtd.h).
    """
    if not isinstance(coeffs, torch.Tensor):
        coeffs = torch.tensor(coeffs, dtype=torch.float64)
    return _Propagate.apply(coeffs, int(n), float(dt), tuple(spacing), int(seg),
                            bool(allow_unstable), *fields)
