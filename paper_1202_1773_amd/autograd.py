"""Differentiable shearlet transform on the GPU.

The forward transform is linear, c = SH f, so its vector-Jacobian product is
the adjoint: d<g, SH f>/df = SH* g (Sec. 3.2-3.3: SH* is the inverse of the
Parseval frame, eq. inverseShearletTransform). `ShearletTransform.backward`
therefore calls the library's adjoint kernels; `ShearletAdjoint` is the
mirror image (its backward is the forward transform). With a complex-
shearlet plan the coefficients are complex and the image real: torch hands
the backward dL/dRe(c) + i dL/dIm(c), whose pull-back to the real image is
Re SH^H g, exactly what the complex adjoint computes.

`l1_denoise` runs plain (sub)gradient descent on
    L(x) = 1/2 ||x - y||^2 + lam ||SH x||_1
with the gradient from autograd, i.e. from the adjoint kernels; for real
shearlets the subgradient lam * sign(SH x) is applied inside the adjoint
kernels (`ShearletL1`).
"""

import torch


class ShearletTransform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, grad_c):
        return ctx.plan.adjoint(grad_c.contiguous()), None


class ShearletAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, plan):
        ctx.plan = plan
        return plan.adjoint(c.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        return ctx.plan.forward(grad_f.contiguous()), None


def shearlet_transform(x, plan):
    """SH x with gradients through the adjoint kernels."""
    return ShearletTransform.apply(x, plan)


def shearlet_adjoint(c, plan):
    """SH* c with gradients through the forward kernels."""
    return ShearletAdjoint.apply(c, plan)


class ShearletL1(torch.autograd.Function):
    """lam * ||SH x||_1 for a real-shearlet plan. Backward: SH*(lam g sign(c))
    in one call of the adjoint kernels, which apply the sign as they read the
    coefficients (the scale lam * g stays on the device)."""

    @staticmethod
    def forward(ctx, x, plan, lam):
        c = plan.forward(x.contiguous())
        ctx.plan, ctx.lam = plan, lam
        ctx.save_for_backward(c)
        return lam * torch.linalg.vector_norm(c, ord=1)

    @staticmethod
    def backward(ctx, g):
        (c,) = ctx.saved_tensors
        scale = (g * ctx.lam).reshape(1).to(torch.float32).contiguous()
        return ctx.plan.adjoint_sign(c, scale), None, None


def shearlet_l1(x, plan, lam):
    """lam * ||SH x||_1 (the modulus of complex coefficients for a
    complex-shearlet plan), differentiable in x."""
    if plan.complex_shearlets:
        return lam * torch.linalg.vector_norm(shearlet_transform(x, plan), ord=1)
    return ShearletL1.apply(x, plan, lam)


def l1_loss(x, y, plan, lam):
    """1/2 ||x - y||^2 + lam ||SH x||_1, summed over the batch. The l1 norm is
    one reduction over the coefficients; its gradient lam * sign(c) is pulled
    back by the adjoint kernels without being stored."""
    return 0.5 * ((x - y) ** 2).sum() + shearlet_l1(x, plan, lam)


def l1_denoise(y, plan, lam=0.05, steps=200, lr=0.5, x0=None):
    """Gradient descent on l1_loss from x0 (default y); returns (x, losses)."""
    x = (y.clone() if x0 is None else x0.clone()).requires_grad_(True)
    losses = []
    for _ in range(steps):
        loss = l1_loss(x, y, plan, lam)
        (g,) = torch.autograd.grad(loss, x)
        with torch.no_grad():
            x -= lr * g
        losses.append(loss.detach())
    return x.detach(), torch.stack(losses)
