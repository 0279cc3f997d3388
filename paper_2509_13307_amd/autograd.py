"""torch.autograd.Function over ns_loglike_grad_batch: the forward call also
computes the hand-written adjoint, and backward scales it by the incoming
gradient, so a gradient-based sampler (HMC) can run on the library."""
import torch


class LogLike(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, model, precision):
        logl, grad = model.loglike_grad(theta.detach(), precision)
        if theta.shape[1] > grad.shape[1]:
            grad = torch.nn.functional.pad(grad, (0, theta.shape[1] - grad.shape[1]))
        ctx.save_for_backward(grad)
        return logl

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g[:, None] * grad, None, None


def loglike(model, theta, precision="fp64"):
    """Differentiable batched log-likelihood logL(theta) [B]."""
    return LogLike.apply(theta, model, precision)
