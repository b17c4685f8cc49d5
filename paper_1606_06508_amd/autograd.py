"""torch.autograd front of the HIP path: r = FhEval.apply(nodes, values, x, d).

The forward pass is fh_eval_forward, which evaluates r and keeps, in its own
workspace, what the adjoint needs per point (1/D, r and the hit data) and,
when x requires a gradient, the derivative r'(x); the backward pass is
fh_eval_backward_saved: dL/dx = grad_r r'(x) and one pass over the (point,
node) pairs for the node sums.  The gradients are
with respect to the values, the evaluation points and the nodes (total
derivative, through the weights).  No gradient flows to d (an integer).
With saved=False the forward is fh_eval and the backward the two-pass
fh_eval_backward (no per-point state kept between the passes).
"""
import torch

from . import fh


class FhEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nodes, values, x, d, precision="fp64", saved=True):
        nodes, values, x = nodes.contiguous(), values.contiguous(), x.contiguous()
        ctx.d = int(d)
        ctx.precision = precision
        if saved:
            r, ctx.state = fh.eval_forward(nodes, values, int(d), x, precision=precision,
                                           derivative=ctx.needs_input_grad[2])
        else:
            r = fh.evaluate(nodes, values, int(d), x, precision=precision)
            ctx.state = None
        ctx.save_for_backward(nodes, values, x)
        return r

    @staticmethod
    def backward(ctx, grad_r):
        nodes, values, x = ctx.saved_tensors
        need_nodes, need_values, need_x = ctx.needs_input_grad[:3]
        if ctx.state is not None:
            gv, gx, gn = fh.eval_backward_saved(ctx.state, grad_r.contiguous(),
                                                need_values=need_values, need_x=need_x,
                                                need_nodes=need_nodes)
        else:
            gv, gx, gn = fh.eval_backward(nodes, values, ctx.d, x, grad_r.contiguous(),
                                          need_values=need_values, need_x=need_x,
                                          need_nodes=need_nodes, precision=ctx.precision)
        return gn, gv, gx, None, None, None


def interpolate(nodes, values, x, d, precision="fp64", saved=True):
    """Differentiable r(x) of the Floater-Hormann interpolant."""
    return FhEval.apply(nodes, values, x, d, precision, saved)
