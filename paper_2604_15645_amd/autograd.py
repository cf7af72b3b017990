"""torch.autograd.Function over the fused residual + gradient step.

forward() makes one pinn_residual_bwd call, which returns the loss and its gradient with
respect to every parameter together; backward() scales that gradient by the incoming
gradient.  Double backward is not supported."""
import torch

from . import binding


class PinnResidualLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, points, fourier_B, net_spec, pde_spec, anchors, prec, tune):
        out = binding.residual_step(net_spec, pde_spec, params.detach(), fourier_B, points,
                                    anchors, prec=prec, grad=True, residual=False, tune=tune)
        ctx.save_for_backward(out["grad"])
        ctx.param_dtype = params.dtype
        return out["loss"][0].to(params.dtype)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout.to(torch.float64) * g).to(ctx.param_dtype), None, None, None, None, None, None, None


def pinn_loss(params, points, fourier_B, net_spec, pde_spec, anchors=(), prec="bf16x3", tune=None):
    """Scalar residual loss whose .backward() deposits dL/dparams into params.grad."""
    return PinnResidualLoss.apply(params, points, fourier_B, net_spec, pde_spec, tuple(anchors),
                                  prec, tune)
