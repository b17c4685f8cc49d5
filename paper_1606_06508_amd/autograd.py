"""torch.autograd front of the HIP path: r = FhEval.apply(nodes, values, x, d).

The forward pass is fh_eval; the backward pass is the adjoint kernel
fh_eval_backward, which returns the gradients with respect to the values,
the evaluation points and the nodes (total derivative, through the
weights).  No gradient flows to d (an integer).
"""
import torch

from . import fh


class FhEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nodes, values, x, d, precision="fp64"):
        r = fh.evaluate(nodes.contiguous(), values.contiguous(), int(d), x.contiguous(),
                        precision=precision)
        ctx.save_for_backward(nodes, values, x)
        ctx.d = int(d)
        ctx.precision = precision
        return r

    @staticmethod
    def backward(ctx, grad_r):
        nodes, values, x = ctx.saved_tensors
        need_nodes, need_values, need_x = ctx.needs_input_grad[:3]
        gv, gx, gn = fh.eval_backward(nodes.contiguous(), values.contiguous(), ctx.d,
                                      x.contiguous(), grad_r.contiguous(),
                                      need_values=need_values, need_x=need_x,
                                      need_nodes=need_nodes, precision=ctx.precision)
        return gn, gv, gx, None, None


def interpolate(nodes, values, x, d, precision="fp64"):
    """Differentiable r(x) of the Floater-Hormann interpolant."""
    return FhEval.apply(nodes, values, x, d, precision)
