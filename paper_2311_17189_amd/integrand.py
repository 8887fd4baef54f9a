"""The integrand of the spatial integrals as a callable (Sec. 5.2): a diagram's
AMI solution bound to its external parameters, evaluated on batches of
internal momenta, and its Monte-Carlo integral over the Brillouin zone.

``Integrand(terms, q, t, mu, ext_freqs, beta)(k)`` maps a float64 CUDA tensor
k [N_E, 2 n_int] (rows of internal momenta, components x, y per loop) to the
integrand out [N_F, N_E] at every external frequency row, as the paper's
integrand class does for an external integrator; ``integrate(n, seed)``
estimates the integral with momenta drawn in the kernel (``amiIntegrateHubbard``).
Every evaluation runs in the library's kernels.
"""
from __future__ import annotations

from ._lib import Terms, evaluate_hubbard, integrate_hubbard, mc_estimate


class Integrand:
    def __init__(self, terms: Terms, q, t: float, mu: float, ext_freqs, beta: float, e_reg: float = 0.0):
        self.terms, self.q, self.t, self.mu = terms, q, t, mu
        self.ext_freqs, self.beta, self.e_reg = ext_freqs, beta, e_reg

    def __call__(self, k, stream=None):
        out, _ = evaluate_hubbard(self.terms, k, self.q, self.t, self.mu, self.ext_freqs, self.beta,
                                  self.e_reg, stream=stream)
        return out

    def integrate(self, n_samples: int, seed: int = 0, stream=None):
        """(mean [N_F] complex, standard error [N_F, 2]) over ``n_samples`` uniform
        momenta; the measure is d^2k/(2 pi)^2 per loop."""
        sums = integrate_hubbard(self.terms, n_samples, seed, self.q, self.t, self.mu, self.ext_freqs,
                                 self.beta, self.e_reg, stream=stream)
        return mc_estimate(sums, n_samples)
