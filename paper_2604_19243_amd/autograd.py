"""torch.autograd binding of the evaluate: the potentials of charges at fixed
points, differentiable in the charges and in the point positions.

Forward is kifmm_evaluate (with the field kept when the positions need a
gradient); backward is kifmm_evaluate_vjp, which runs the adjoint evaluate and
the combination on the device.  This module only marshals arguments: no step of
the computation runs in torch.  The octree is built once from the positions, so
the derivative in the positions is that of the evaluate for points that stay in
their leaves.
"""

import numpy as np
import torch

from . import kifmm


class DifferentiableFMM:
    """Tree, operators and a plan with KIFMM_VJP for one point set on one device."""

    def __init__(self, points, depth, p, cube=None, eps_pinv=1e-7, eps_svd=1e-6, m2l_flags=0, stream=None):
        """points: host [n,3] float32 array, or a [n,3] float32 device tensor (the tree is then built
        from device memory, on `stream`, and the plan lives on that tensor's device)."""
        if isinstance(points, torch.Tensor):
            pts = points.detach().to(torch.float32).contiguous()
            if not pts.is_cuda:
                pts = pts.numpy()
        else:
            pts = np.ascontiguousarray(points, dtype=np.float32)
        flags = kifmm.KIFMM_POTENTIAL | kifmm.KIFMM_GRADIENT | kifmm.KIFMM_VJP | m2l_flags
        self.fmm = kifmm.FMM(pts, depth, p, cube=cube, eps_pinv=eps_pinv, eps_svd=eps_svd, flags=flags,
                             stream=stream)
        self.n = self.fmm.n

    def close(self):
        self.fmm.close()


class _Potential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, charges, dfmm):
        n = dfmm.n
        if charges.shape != (n,) or charges.dtype != torch.float32 or not charges.is_cuda:
            raise ValueError("charges must be a float32 device tensor of shape [n]")
        if points.shape != (n, 3):
            raise ValueError("points must have shape [n, 3] (the positions the tree was built from)")
        s = charges.detach().contiguous()
        stream = torch.cuda.current_stream(s.device).cuda_stream
        pot = torch.empty(n, device=s.device, dtype=torch.float32)
        field = torch.empty(n, 3, device=s.device, dtype=torch.float32) if ctx.needs_input_grad[0] else None
        dfmm.fmm.evaluate(s, pot, field, stream)
        ctx.dfmm = dfmm
        ctx.save_for_backward(s, field if field is not None else torch.empty(0, device=s.device))
        ctx.has_field = field is not None
        return pot

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_pot):
        s, field = ctx.saved_tensors
        n = ctx.dfmm.n
        w = grad_pot.detach().to(torch.float32).contiguous()
        gc = torch.empty(n, device=s.device, dtype=torch.float32) if ctx.needs_input_grad[1] else None
        gp = torch.empty(n, 3, device=s.device, dtype=torch.float32) if ctx.needs_input_grad[0] else None
        if gc is None and gp is None:
            return None, None, None
        stream = torch.cuda.current_stream(s.device).cuda_stream
        ctx.dfmm.fmm.vjp(s, w, field if ctx.has_field else None, gc, gp, stream)
        return gp, gc, None


def potential(dfmm, points, charges):
    """Potentials f_i = sum_{j != i} s_j / |x_i - x_j| (FMM), differentiable in
    `points` ([n, 3], the positions `dfmm` was built from) and `charges` ([n])."""
    return _Potential.apply(points, charges, dfmm)
