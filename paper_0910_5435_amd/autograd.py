"""Differentiable synthesis: a torch.autograd.Function over the butterfly transform.

Synthesis is linear in the coefficients, f = S beta, so for a real loss the gradient with
respect to the coefficients is the adjoint S^H applied to the gradient with respect to the
grid.  S^H is the transposed butterfly with the node weights left out, the same factors
read in the other orientation (the transposition remark after the description of the
butterfly algorithm, Section 3.2); the library computes it with ``sht_synth_adjoint``:

* complex fields: gamma_k^m = sum_i Pbar_k^|m|(x_i) sum_j g_ij e^{-i m phi_j}, which is the
  gradient in PyTorch's convention for complex leaves (d/dRe + i d/dIm);
* real fields (m >= 0 stored, beta^{-m} = conj(beta^m)): the same sum doubled for m > 0,
  and its real part at m = 0, where the imaginary part of beta does not enter synthesis.

Forward and backward both run in the library's kernels in the precision asked for
(``split32`` by default: the split-FP32 matrix-core form).
"""
from .sht import Plan

__all__ = ["SynthFunction", "synth"]


def _torch():
    import torch

    return torch


class SynthFunction(_torch().autograd.Function):
    """grid = synth(coeff); backward: coeff_grad = synth_adjoint(grid_grad)."""

    @staticmethod
    def forward(ctx, coeff, plan, precision):
        ctx.plan = plan
        ctx.precision = precision
        return plan.synth(coeff.detach().contiguous(), precision=precision)

    @staticmethod
    def backward(ctx, grad_grid):
        if not ctx.needs_input_grad[0]:
            return None, None, None
        g = grad_grid.contiguous()
        return ctx.plan.synth_adjoint(g, precision=ctx.precision), None, None


def synth(coeff, plan: Plan, precision="split32"):
    """Differentiable synthesis of coefficients (F, n_coeffs) complex128 on the device."""
    return SynthFunction.apply(coeff, plan, precision)

