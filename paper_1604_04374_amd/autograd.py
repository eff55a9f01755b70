"""torch.autograd support: the expansion as a differentiable function of the
signal and of the spectra of its impulse responses.

Forward runs ``pc_apply``; backward runs the hand-written adjoint
(``pc_apply_adjoint``) for the signal and ``pc_grad_spectra`` for the
spectra.  Spectra use the natural layout of a real FFT (``torch.fft.rfft`` /
``rfft2``), complex64.
"""
from __future__ import annotations

import torch

from . import Plan

__all__ = ["ExpansionFunction", "expansion", "ExpansionOperator"]


def _load(plan: Plan, spec: torch.Tensor):
    # Import only when the plan last saw a different tensor or an older
    # version of this one.  The plan keeps a reference to the tensor it saw,
    # so a new tensor can never be mistaken for it by address.
    last = getattr(plan, "_spec_seen", None)
    if last is None or last[0] is not spec or last[1] != spec._version:
        plan.set_spectra(spec.detach())
        plan._spec_seen = (spec, spec._version)


class ExpansionFunction(torch.autograd.Function):
    """``y = H_m u`` with ``H_m`` given by ``plan`` and the spectra ``spec``."""

    @staticmethod
    def forward(ctx, u, spec, plan):
        _load(plan, spec)
        y = plan.apply(u.contiguous())
        ctx.plan = plan
        ctx.save_for_backward(u, spec)
        return y

    @staticmethod
    def backward(ctx, gy):
        u, spec = ctx.saved_tensors
        plan = ctx.plan
        _load(plan, spec)
        gy = gy.contiguous()
        gu = plan.apply_adjoint(gy) if ctx.needs_input_grad[0] else None
        gs = plan.grad_spectra(u.contiguous(), gy) if ctx.needs_input_grad[1] else None
        return gu, gs, None


def expansion(u, spec, plan):
    return ExpansionFunction.apply(u, spec, plan)


class ExpansionOperator(torch.nn.Module):
    """A convolution-product operator (or, with ``product_convolution=True``,
    a product-convolution operator, eq. 1.3) whose spectra are trainable.

    ``windows``/``h`` as for :class:`Plan`; the initial spectra are the plan's
    transform of ``h``.
    """

    def __init__(self, windows, h, batch=1, product_convolution=False):
        super().__init__()
        self.plan = Plan(windows, h, batch=batch, gradients=True, product_convolution=product_convolution)
        self.spec = torch.nn.Parameter(self.plan.get_spectra())
        torch.cuda.synchronize()

    def forward(self, u):
        return ExpansionFunction.apply(u, self.spec, self.plan)
