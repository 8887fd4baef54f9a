"""Pins of the oracle's Monte-Carlo path (oracle/mc.py): the counter-based
generator against its published known-answer vectors, the sample mapping,
and the estimate against a deterministic quadrature of the same integral."""
import os

import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, order2_example
from oracle.evaluate import energies_from_k, evaluate_terms
from oracle.mc import draw_momenta, mc_sums, philox4x32, philox4x32_vec

from parity import oracle_terms

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in _kat():
        assert philox4x32(ctr, key) == want


def test_philox_vectorized_equals_scalar():
    rng = np.random.default_rng(60)
    c = rng.integers(0, 2 ** 32, size=(4, 50), dtype=np.uint64)
    k0, k1 = 0x12345678, 0x9abcdef0
    got = philox4x32_vec(c[0], c[1], c[2], c[3], k0, k1)
    for j in range(50):
        assert [int(g[j]) for g in got] == philox4x32([int(x[j]) for x in c], [k0, k1])


def test_draw_momenta_layout_and_range():
    k = draw_momenta(10, 2000, 8, seed=(7 << 32) | 3)
    assert k.shape == (2000, 8) and np.all(np.abs(k) < np.pi)
    # sample 10 + j uses counter (10 + j, 0, b, 0): recompute one row by hand
    w = philox4x32([15, 0, 0, 0], [3, 7]) + philox4x32([15, 0, 1, 0], [3, 7])
    want = [((x + 0.5) * 2.0 ** -32 - 0.5) * 2 * np.pi for x in w]
    assert k[5].tolist() == want
    # uniform on (-pi, pi): mean and variance of 16000 values
    assert abs(k.mean()) < 4 * np.pi / np.sqrt(3 * k.size)
    assert abs(k.var() - np.pi ** 2 / 3) < 0.05


def test_mc_estimate_matches_quadrature():
    """Order 2 (four momentum components): the Monte-Carlo mean over 2^16
    draws against the periodic trapezoid rule on a 14^4 grid of the same
    integrand (analytic and periodic in k, so the rule converges
    exponentially), within four standard errors."""
    d = order2_example()
    terms = oracle_terms(d)
    beta, t, mu = 2.0, 1.0, 0.3
    q = np.array(DEFAULT_Q)
    w = np.array([1j * np.pi / beta])
    n = 1 << 16
    s = mc_sums(terms, d.alpha, d.n_int, n, seed=11, q=q, t=t, mu=mu, ext_freqs=w, beta=beta)
    mean = (s[0, 0] + 1j * s[0, 1]) / n
    err_re = np.sqrt((s[0, 2] / n - (s[0, 0] / n) ** 2) / n)
    err_im = np.sqrt((s[0, 3] / n - (s[0, 1] / n) ** 2) / n)
    g = -np.pi + 2 * np.pi * np.arange(14) / 14
    grid = np.stack(np.meshgrid(g, g, g, g, indexing="ij"), axis=-1).reshape(-1, 4)
    E = energies_from_k(d.alpha, grid, q, t, mu, dtype=np.float64)
    quad = evaluate_terms(terms, d.n_int, E, w, beta, dtype=np.float64).astype(np.complex128).mean()
    assert abs(mean.real - quad.real) < 4 * err_re
    assert abs(mean.imag - quad.imag) < 4 * err_im
    # and the sums are the plain sums of the drawn samples' values
    k = draw_momenta(0, 1000, 4, seed=11)
    v = evaluate_terms(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu, dtype=np.float64), w, beta,
                       dtype=np.float64).astype(np.complex128)
    s1 = mc_sums(terms, d.alpha, d.n_int, 1000, seed=11, q=q, t=t, mu=mu, ext_freqs=w, beta=beta, chunk=300)
    np.testing.assert_allclose(s1[0], [v.real.sum(), v.imag.sum(), (v.real ** 2).sum(), (v.imag ** 2).sum()],
                               rtol=1e-13)
