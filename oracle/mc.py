"""Monte-Carlo integration over the internal momenta (Sec. 5.2): the spatial
integral of the AMI integrand estimated by the mean over uniformly drawn
wavevectors, with the row average of Sec. 2.3.  TEST INFRASTRUCTURE ONLY.

The momenta are drawn from a counter-based generator, so that the library and
this module draw the same samples without exchanging them: Philox4x32 with 10
rounds (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11), written here from its published definition.

Sample s of a run with 64-bit seed S takes the words of the blocks
``philox((s mod 2^32, s div 2^32, b, 0), (S mod 2^32, S div 2^32))`` for
b = 0, 1, ... in order; component c of k (c < d*n_int, row-major as the k_int
matrix of Sec. 5.2) uses word c and is ``k_c = (u_c - 1/2) * 2 pi`` with
``u_c = (word + 1/2) / 2^32`` -- uniform on (-pi, pi), every step exact in
float64 except the final product.
"""
from __future__ import annotations

import numpy as np

from .evaluate import energies_from_k, evaluate_terms

# Philox4x32 constants of the published definition: the two round multipliers
# and the Weyl increments of the key schedule
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
TWO_PI = 2.0 * np.pi


def philox4x32(counter, key, rounds: int = 10):
    """One Philox4x32 block: four 32-bit words from a 4-word counter and a
    2-word key (plain Python integers).  Each round multiplies words 0 and 2
    by the two constants (full 64-bit products), and the new words are
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key grows by the Weyl
    increments after every round."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in counter)
    k0, k1 = (int(x) & MASK32 for x in key)
    for _ in range(rounds):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK32, p1 & MASK32, ((p0 >> 32) ^ c3 ^ k1) & MASK32, p0 & MASK32
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return [c0, c1, c2, c3]


def philox4x32_vec(c0, c1, c2, c3, k0: int, k1: int, rounds: int = 10):
    """:func:`philox4x32` over numpy arrays of counters (uint64 arithmetic)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & np.uint64(MASK32) for x in (c0, c1, c2, c3))
    m32 = np.uint64(MASK32)
    for _ in range(rounds):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        n0 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0)) & m32
        n2 = ((p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1)) & m32
        c0, c1, c2, c3 = n0, p1 & m32, n2, p0 & m32
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return c0, c1, c2, c3


def draw_momenta(first: int, count: int, n_comp: int, seed: int) -> np.ndarray:
    """Momenta of samples first .. first+count-1, float64 [count, n_comp]."""
    s = np.arange(first, first + count, dtype=np.uint64)
    lo, hi = s & np.uint64(MASK32), s >> np.uint64(32)
    k0, k1 = seed & MASK32, (seed >> 32) & MASK32
    words = []
    for b in range((n_comp + 3) // 4):
        words.extend(philox4x32_vec(lo, hi, np.full_like(s, b), np.zeros_like(s), k0, k1))
    w = np.stack(words[:n_comp], axis=1).astype(np.float64)
    u = (w + 0.5) * 2.0 ** -32
    return (u - 0.5) * TWO_PI


def mc_sums(terms, alpha, n_int: int, n_samples: int, seed: int, q, t, mu, ext_freqs, beta,
            e_reg=0.0, dim: int = 2, chunk: int = 4096, dtype=np.float64):
    """Sums over the samples of the integrand at every frequency row:
    ``[n_f, 4]`` = (sum Re I, sum Im I, sum (Re I)^2, sum (Im I)^2).  The mean
    is the Monte-Carlo estimate of the integral over the Brillouin zone (with
    the measure d^dk/(2 pi)^d per loop), sum/n; its variance follows from the
    squares."""
    w = np.asarray(ext_freqs)
    n_f = w.shape[0]
    acc = np.zeros((n_f, 4))
    for first in range(0, n_samples, chunk):
        cnt = min(chunk, n_samples - first)
        k = draw_momenta(first, cnt, dim * n_int, seed)
        E = energies_from_k(alpha, k, q, t, mu, dim, dtype)
        v = evaluate_terms(terms, n_int, E, w, beta, e_reg, dtype=dtype).astype(np.complex128)
        acc[:, 0] += v.real.sum(axis=1)
        acc[:, 1] += v.imag.sum(axis=1)
        acc[:, 2] += (v.real ** 2).sum(axis=1)
        acc[:, 3] += (v.imag ** 2).sum(axis=1)
    return acc
