"""PyTorch autograd view of the gauge action (Wilson, or improved with
rectangle coefficient c1).

S(omega) = S_G(exp(omega) U0), with omega a field of su(3) components
(shape (4, V, 8), the momentum layout), is differentiated in the chart at
omega = 0, where every derivative is a kernel of the library:

  S(0)                     fgi_improved_gauge_action
  dS/domega (0) = -F_G     fgi_force (no fermions) (Section 4: the force is
                                                    minus the e_a derivative)
  H v = (e_a e_b + e_b e_a) S v / 2 = -J_v[F_G] + [v, F_G] / 2
                           fgi_improved_gauge_hvp (along v = F_G this is the
                                                    Section 4 force gradient)

Only omega = 0 is supported (the chart is re-centred on U0 for every call);
a non-zero omega raises, because the derivatives of the exponential map
would then enter.
"""
import torch

from . import fgi


def _check_zero(omega):
    if bool(torch.any(omega != 0)):
        raise ValueError("GaugeAction is evaluated in the chart at omega = 0; re-centre U0 instead")


class _GaugeGrad(torch.autograd.Function):
    """omega -> dS/domega = -F_G(U0) at omega = 0; its backward is H v."""

    @staticmethod
    def forward(fctx, omega, U0, beta, c1, dims, ctx):
        fctx.save_for_backward(U0)
        fctx.beta, fctx.c1, fctx.dims, fctx.ctx = beta, c1, dims, ctx
        F, _ = ctx.force(dims, fgi.Action(beta=beta, c1=c1), U0)
        return -F

    @staticmethod
    def backward(fctx, v):
        (U0,) = fctx.saved_tensors
        hv = fctx.ctx.improved_gauge_hvp(fctx.dims, fctx.beta, fctx.c1, U0, v.contiguous())
        return hv, None, None, None, None, None


class GaugeAction(torch.autograd.Function):
    """S_G(exp(omega) U0) as a differentiable scalar of omega (at omega = 0)."""

    @staticmethod
    def forward(fctx, omega, U0, beta, c1, dims, ctx):
        _check_zero(omega)
        fctx.save_for_backward(omega, U0)
        fctx.beta, fctx.c1, fctx.dims, fctx.ctx = beta, c1, dims, ctx
        S = ctx.improved_gauge_action(dims, beta, c1, U0)
        return torch.tensor(S, dtype=torch.float64, device=omega.device)

    @staticmethod
    def backward(fctx, g):
        omega, U0 = fctx.saved_tensors
        grad = _GaugeGrad.apply(omega, U0, fctx.beta, fctx.c1, fctx.dims, fctx.ctx)
        return g * grad, None, None, None, None, None


def gauge_action(ctx, dims, beta, U0, omega, c1=0.0):
    """Differentiable S_G(exp(omega) U0) (rectangle coefficient c1, 0 = Wilson);
    omega must be all zeros."""
    return GaugeAction.apply(omega, U0, beta, float(c1), tuple(dims), ctx)
