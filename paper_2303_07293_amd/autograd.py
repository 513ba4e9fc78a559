"""torch.autograd binding of the differentiable stacked S/N.

The forward pass and its hand-written adjoint both run in the library's
refinement kernel (`sst_refine` with zero ascent steps returns SN and
dSN/dtheta together); backward only scales that gradient by the incoming
one.  Frames, timestamps and the PSF are constants of the objective.
"""

from __future__ import annotations

from .binding import sst_refine


def _autograd_function():
    import torch

    class StackedSNR(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, frames, t, t_ref, cutout, fwhm, scale):
            _, snr, grad = sst_refine(frames, t, t_ref, params.detach().float().contiguous(), cutout=cutout,
                                      fwhm=fwhm, steps=0, scale=scale)
            ctx.save_for_backward(grad)
            return snr

        @staticmethod
        def backward(ctx, grad_snr):
            (grad,) = ctx.saved_tensors
            return grad_snr[:, None] * grad, None, None, None, None, None, None

    return StackedSNR


class _Lazy:
    fn = None


def StackedSNR():  # noqa: N802 - returns the torch.autograd.Function class
    if _Lazy.fn is None:
        _Lazy.fn = _autograd_function()
    return _Lazy.fn


def stacked_snr(params, frames, t, t_ref: float, cutout: int = 33, fwhm: float = 2.5, scale=None):
    """Differentiable SN(theta) for params [n_cand][4] = (x0, y0, vx, vy)."""
    return StackedSNR().apply(params, frames, t, t_ref, cutout, fwhm, scale)
