"""``torch.autograd.Function`` wrappers: forward through ``amiEvaluate*``,
backward through ``amiEvaluate*Adjoint`` (both HIP kernels of libamigpu)."""
from __future__ import annotations

import torch

from ._lib import (Terms, evaluate, evaluate_adjoint, evaluate_hubbard,
                   evaluate_hubbard_adjoint)


class AmiEvaluate(torch.autograd.Function):
    """``(out [N_F, N_E], out_sum [N_F]) = AmiEvaluate.apply(terms, energies,
    ext_freqs, beta, e_reg)`` with gradients for the energies (float64
    [N_E, nE]), the external frequencies (complex128 [N_F, n_ext]) and beta (a
    0-dim float64 tensor), at fixed e_reg."""

    @staticmethod
    def forward(ctx, terms: Terms, energies, ext_freqs, beta, e_reg: float = 0.0):
        out, out_sum = evaluate(terms, energies.detach(), ext_freqs.detach(), float(beta), e_reg,
                                want_out=True, want_sum=True)
        ctx.terms = terms
        ctx.e_reg = e_reg
        ctx.save_for_backward(energies, ext_freqs, torch.as_tensor(beta, dtype=torch.float64))
        return out, out_sum

    @staticmethod
    def backward(ctx, grad_out, grad_sum):
        energies, ext_freqs, beta = ctx.saved_tensors
        g_e, g_b, g_w = evaluate_adjoint(ctx.terms, energies.detach(), ext_freqs.detach(),
                                         float(beta), ctx.e_reg, grad_out=grad_out, grad_sum=grad_sum)
        g_w = g_w.reshape(ext_freqs.shape)
        return None, g_e, g_w, g_b.to(beta.device) if ctx.needs_input_grad[3] else None, None


class AmiHubbard(torch.autograd.Function):
    """``(out, out_sum) = AmiHubbard.apply(terms, k, q, t, mu, ext_freqs, beta,
    e_reg)``: energies from momenta in the kernel (Sec. 5.2); gradients for k
    (float64 [N_E, 2 n_int]), t, mu, beta (0-dim float64 tensors) and the
    external frequencies."""

    @staticmethod
    def forward(ctx, terms: Terms, k, q, t, mu, ext_freqs, beta, e_reg: float = 0.0):
        out, out_sum = evaluate_hubbard(terms, k.detach(), q, float(t), float(mu), ext_freqs.detach(),
                                        float(beta), e_reg, want_out=True, want_sum=True)
        ctx.terms = terms
        ctx.q = q
        ctx.e_reg = e_reg
        ctx.save_for_backward(k, ext_freqs, torch.as_tensor(t, dtype=torch.float64),
                              torch.as_tensor(mu, dtype=torch.float64),
                              torch.as_tensor(beta, dtype=torch.float64))
        return out, out_sum

    @staticmethod
    def backward(ctx, grad_out, grad_sum):
        k, ext_freqs, t, mu, beta = ctx.saved_tensors
        g_k, g_mu, g_t, g_b, g_w = evaluate_hubbard_adjoint(
            ctx.terms, k.detach(), ctx.q, float(t), float(mu), ext_freqs.detach(), float(beta),
            ctx.e_reg, grad_out=grad_out, grad_sum=grad_sum)
        return (None, g_k, None, g_t, g_mu, g_w.reshape(ext_freqs.shape), g_b, None)
