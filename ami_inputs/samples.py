"""Seeded sample generators: momenta, energies, external frequencies.

* Momenta ``k`` for the Monte-Carlo example of Sec. 5.2: every internal
  momentum uniform in the Brillouin zone ``[-pi, pi)^d``, laid out as the
  ``N_E x (d*m)`` matrix of Sec. 5.2 (components of the first loop momentum,
  then the second, ...).
* Uniform energies on ``(-a, a)`` as in the evaluation example of Sec. 5.1.3.
* Fermionic Matsubara frequencies ``i(2j+1)pi/beta`` (Sec. 5.1.3) and a
  real-frequency grid ``omega + i*Gamma`` for the continuation of Sec. 1.

Only random numbers and plain grids are produced here.
"""
from __future__ import annotations

import numpy as np

# external momentum used with the Hubbard dispersion: the nodal Fermi point at mu = 0
DEFAULT_Q = (np.pi / 2, np.pi / 2)


def k_samples(n_e: int, n_int: int, seed, dim: int = 2) -> np.ndarray:
    """float64 [n_e, dim*n_int], each component uniform in [-pi, pi)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n_e, dim * n_int))
    return (2.0 * np.pi) * u - np.pi


def uniform_energies(n_e: int, n_eps: int, seed, a: float = 8.0) -> np.ndarray:
    """float64 [n_e, n_eps], uniform on (-a, a) (the example of Sec. 5.1.3)."""
    rng = np.random.default_rng(seed)
    return 2.0 * a * rng.random((n_e, n_eps)) - a


def complex_energies(n_e: int, n_eps: int, seed, a: float = 3.0, eta: float = 0.1) -> np.ndarray:
    """complex128 [n_e, n_eps]: real parts uniform on (-a, a), imaginary parts
    uniform on (-eta, eta) (energies with a broadening; the energy vector's
    element type is complex, Sec. 5.1.3)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-a, a, (n_e, n_eps)) + 1j * rng.uniform(-eta, eta, (n_e, n_eps))


def matsubara_freqs(n_f: int, beta: float, first: int = 0) -> np.ndarray:
    """complex128 [n_f]: i*(2j+1)*pi/beta for j = first .. first+n_f-1."""
    j = np.arange(first, first + n_f, dtype=np.float64)
    return 1j * (2.0 * j + 1.0) * np.pi / beta


def real_freqs(n_f: int, lo: float, hi: float, gamma: float) -> np.ndarray:
    """complex128 [n_f]: omega + i*gamma on an even grid omega in [lo, hi]."""
    return np.linspace(lo, hi, n_f) + 1j * gamma
