"""``torch.autograd.Function`` wrappers: forward through ``amiEvaluate*``,
backward through ``amiEvaluate*Adjoint`` (both HIP kernels of libamigpu).

The scalars beta, t and mu reach the kernels by value.  They may be Python
numbers or 0-dim tensors; a tensor's value is read once, in the forward, and
kept on the context, so the backward reads no device value back.  A CPU
tensor (or a number) costs no host synchronization at all, and the calls can
then be captured in a HIP graph; a CUDA tensor costs one read in the forward.
Gradients are returned only for tensor inputs that require them, on each
input's own device."""
from __future__ import annotations

import torch

from ._lib import (Terms, evaluate, evaluate_adjoint, evaluate_complex, evaluate_complex_adjoint,
                   evaluate_hubbard, evaluate_hubbard_adjoint)


def _value(x) -> float:
    return float(x.detach().item()) if isinstance(x, torch.Tensor) else float(x)


def _meta(x):
    """(shape, device, dtype) of a tensor input, None for a number."""
    return (x.shape, x.device, x.dtype) if isinstance(x, torch.Tensor) else None


def _grad_for(ctx, i, meta, g):
    """Gradient g for input i, shaped and placed like it, or None when the
    input is a number or needs no gradient."""
    if not ctx.needs_input_grad[i] or meta is None:
        return None
    shape, device, dtype = meta
    return g.reshape(shape).to(device=device, dtype=dtype)


class AmiEvaluate(torch.autograd.Function):
    """``(out [N_F, N_E], out_sum [N_F]) = AmiEvaluate.apply(terms, energies,
    ext_freqs, beta, e_reg)`` with gradients for the energies (float64
    [N_E, nE]), the external frequencies (complex128 [N_F, n_ext]) and beta (a
    number or a 0-dim float64 tensor), at fixed e_reg."""

    @staticmethod
    def forward(ctx, terms: Terms, energies, ext_freqs, beta, e_reg: float = 0.0):
        b = _value(beta)
        out, out_sum = evaluate(terms, energies.detach(), ext_freqs.detach(), b, e_reg,
                                want_out=True, want_sum=True)
        ctx.terms = terms
        ctx.e_reg = e_reg
        ctx.beta = b
        ctx.beta_meta = _meta(beta)
        ctx.save_for_backward(energies, ext_freqs)
        return out, out_sum

    @staticmethod
    def backward(ctx, grad_out, grad_sum):
        energies, ext_freqs = ctx.saved_tensors
        g_e, g_b, g_w = evaluate_adjoint(ctx.terms, energies.detach(), ext_freqs.detach(),
                                         ctx.beta, ctx.e_reg, grad_out=grad_out, grad_sum=grad_sum)
        return (None, g_e if ctx.needs_input_grad[1] else None,
                g_w.reshape(ext_freqs.shape) if ctx.needs_input_grad[2] else None,
                _grad_for(ctx, 3, ctx.beta_meta, g_b), None)


class AmiEvaluateComplex(torch.autograd.Function):
    """``(out [N_F, N_E], out_sum [N_F]) = AmiEvaluateComplex.apply(terms,
    energies, ext_freqs, beta, e_reg)`` at complex energies (complex128
    [N_E, nE], Sec. 5.1.3), with gradients for the energies and the external
    frequencies in torch's convention for complex inputs (dL/dRe + i dL/dIm,
    which is what amiEvaluateComplexAdjoint returns) and for beta, at fixed
    e_reg."""

    @staticmethod
    def forward(ctx, terms: Terms, energies, ext_freqs, beta, e_reg: float = 0.0):
        b = _value(beta)
        out, out_sum = evaluate_complex(terms, energies.detach(), ext_freqs.detach(), b, e_reg,
                                        want_out=True, want_sum=True)
        ctx.terms = terms
        ctx.e_reg = e_reg
        ctx.beta = b
        ctx.beta_meta = _meta(beta)
        ctx.save_for_backward(energies, ext_freqs)
        return out, out_sum

    @staticmethod
    def backward(ctx, grad_out, grad_sum):
        energies, ext_freqs = ctx.saved_tensors
        g_e, g_b, g_w = evaluate_complex_adjoint(ctx.terms, energies.detach(), ext_freqs.detach(), ctx.beta,
                                                 ctx.e_reg, grad_out=grad_out, grad_sum=grad_sum)
        return (None, g_e if ctx.needs_input_grad[1] else None,
                g_w.reshape(ext_freqs.shape) if ctx.needs_input_grad[2] else None,
                _grad_for(ctx, 3, ctx.beta_meta, g_b), None)


class AmiHubbard(torch.autograd.Function):
    """``(out, out_sum) = AmiHubbard.apply(terms, k, q, t, mu, ext_freqs, beta,
    e_reg)``: energies from momenta in the kernel (Sec. 5.2); gradients for k
    (float64 [N_E, 2 n_int]), the external frequencies, and t, mu, beta when
    they are tensors (numbers or 0-dim float64 tensors)."""

    @staticmethod
    def forward(ctx, terms: Terms, k, q, t, mu, ext_freqs, beta, e_reg: float = 0.0):
        tv, mv, bv = _value(t), _value(mu), _value(beta)
        out, out_sum = evaluate_hubbard(terms, k.detach(), q, tv, mv, ext_freqs.detach(), bv, e_reg,
                                        want_out=True, want_sum=True)
        ctx.terms = terms
        ctx.q = q
        ctx.e_reg = e_reg
        ctx.vals = (tv, mv, bv)
        ctx.scalars = tuple(_meta(x) for x in (t, mu, beta))
        ctx.save_for_backward(k, ext_freqs)
        return out, out_sum

    @staticmethod
    def backward(ctx, grad_out, grad_sum):
        k, ext_freqs = ctx.saved_tensors
        tv, mv, bv = ctx.vals
        g_k, g_mu, g_t, g_b, g_w = evaluate_hubbard_adjoint(
            ctx.terms, k.detach(), ctx.q, tv, mv, ext_freqs.detach(), bv,
            ctx.e_reg, grad_out=grad_out, grad_sum=grad_sum)
        t_in, mu_in, b_in = ctx.scalars
        return (None, g_k if ctx.needs_input_grad[1] else None, None,
                _grad_for(ctx, 3, t_in, g_t), _grad_for(ctx, 4, mu_in, g_mu),
                g_w.reshape(ext_freqs.shape) if ctx.needs_input_grad[5] else None,
                _grad_for(ctx, 6, b_in, g_b), None)
