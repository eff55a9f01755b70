"""torch.autograd support: the expansion as a differentiable function of the
signal and of the spectra of its impulse responses.

Forward runs ``pc_apply_save`` (which leaves in the plan what the backward
pass reuses); backward runs ``pc_backward``: the hand-written adjoint for the
signal and the spectra gradient, from one transform of the output gradient.
Spectra use the natural layout of a real FFT (``torch.fft.rfft`` /
``rfft2``), complex64; a sectioned plan's parameters are its sections'
spectra, concatenated (``Plan.sections``).
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
        u = u.contiguous()
        y = plan.apply_save(u)
        ctx.plan = plan
        ctx.save_for_backward(u, spec)
        return y

    @staticmethod
    def backward(ctx, gy):
        # autograd raises before this point if u was modified in place since
        # the forward, so the plan may reuse what the forward left
        u, spec = ctx.saved_tensors
        plan = ctx.plan
        _load(plan, spec)
        gu, gs = plan.backward(u, gy.contiguous(), want_u=ctx.needs_input_grad[0],
                               want_spectra=ctx.needs_input_grad[1], use_saved=True)
        return gu, gs, None


def expansion(u, spec, plan):
    return ExpansionFunction.apply(u, spec, plan)


class ExpansionOperator(torch.nn.Module):
    """A convolution-product operator (or, with ``product_convolution=True``,
    a product-convolution operator, eq. 1.3) whose spectra are trainable.

    ``windows``/``h`` as for :class:`Plan`; the initial spectra are the plan's
    transform of ``h`` (for a sectioned plan, its sections' spectra).
    ``full_grid`` keeps a 2D operator on the full grid; ``budget`` (bytes)
    bounds the windowed spectra the plan keeps from forward to backward.
    """

    def __init__(self, windows, h, batch=1, product_convolution=False, full_grid=False, budget=None):
        super().__init__()
        self.plan = Plan(windows, h, batch=batch, gradients=True, product_convolution=product_convolution,
                         full_grid=full_grid)
        if budget is not None:
            self.plan.set_budget(budget)
        self.spec = torch.nn.Parameter(self.plan.get_spectra())
        torch.cuda.synchronize()

    def forward(self, u):
        return ExpansionFunction.apply(u, self.spec, self.plan)
