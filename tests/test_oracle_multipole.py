"""Pins of the oracle's poles of higher order (Eq. (5)): the Taylor-coefficient
leaves against high-precision differentiation, the construction against the
plain definition Eq. (1) (truncated Matsubara sums) for a double pole present
from the start and for one that appears only after a first sum, and the
simple-pole solutions unchanged by the option."""
import mpmath as mp
import numpy as np
import pytest

from ami_inputs import random_self_energy
from oracle.brute import brute_force
from oracle.construct import MultipoleError, canonical, construct, serialize
from oracle.evaluate import evaluate_terms, leaf_coefficient


@pytest.mark.parametrize("sigma", [1, -1])
@pytest.mark.parametrize("j", [1, 2, 3])
def test_taylor_leaves_against_mpmath(sigma, j):
    mp.mp.dps = 40
    beta = 2.5
    for x in (-3.1, -0.7, 0.35, 1.9, 6.0):
        f = lambda u: 1 / (sigma * mp.exp(beta * u) + 1)
        want = mp.diff(f, mp.mpf(x), j) / mp.factorial(j)
        got = leaf_coefficient(sigma * (1 + j), np.longdouble(x), np.longdouble(beta))
        assert abs(float(got) - float(want)) <= 1e-15 * abs(float(want)) + 1e-300, (x, got, want)


def _oracle_value(alpha, eps, n_int, fermionic, E, w, beta):
    terms = canonical(construct(alpha, eps, n_int, fermionic, multipole=True))
    return complex(evaluate_terms(terms, n_int, np.array([E]), np.array([w]), beta)[0, 0]), terms


def test_double_pole_single_sum_against_brute_force():
    """(1/beta) sum_nu 1/((i nu + E1)^2 (i nu + i Omega + E2)), bosonic Omega."""
    alpha = np.array([[1, 0], [1, 0], [1, 1]])
    eps = np.array([[1, 0], [1, 0], [0, 1]])
    fermionic = [1, 0]
    beta = 2.0
    with pytest.raises(MultipoleError):
        construct(alpha, eps, 1, fermionic)
    for E, Om in (((0.37, -1.21), 2 * np.pi / beta), ((-0.8, 0.45), 4 * np.pi / beta)):
        w = 1j * Om
        got, terms = _oracle_value(alpha, eps, 1, fermionic, E, [w], beta)
        assert any(abs(code) == 2 for _, leaves, _ in terms for code, _ in leaves)
        # the terms hold one or two denominators: the extended stream
        stream = serialize(terms, 1, 2, 2)
        assert stream[3] == -len(terms) and sorted({len(d) for _, _, d in terms}) == [1, 2]
        ref = brute_force(alpha, eps, 1, E, [w], beta)
        assert abs(got - ref) <= 1e-8 * abs(ref), (got, ref)
        # and the residues written out by hand: T_1 = beta f'(beta x) at x = -E1
        f = lambda y: 1 / (np.exp(y) + 1)
        x0, d = -E[0], 1j * Om + E[1] - E[0]
        fp = -f(beta * x0) * f(-beta * x0)
        closed = beta * fp / d - f(beta * x0) / d ** 2 + f(-beta * E[1]) / d ** 2
        assert abs(got - closed) <= 1e-12 * abs(closed)


def test_double_pole_after_a_first_sum_against_brute_force():
    """A = nu1 + E1, B = nu2 + w + E2, C = nu2 - nu1 + w + E2 - E1: the residue
    of the first sum at A's pole turns C into B, a double pole in nu2."""
    alpha = np.array([[1, 0, 0], [0, 1, 1], [-1, 1, 1]])
    eps = np.array([[1, 0], [0, 1], [-1, 1]])
    fermionic = [1, 1, 0]
    beta = 1.5
    with pytest.raises(MultipoleError):
        construct(alpha, eps, 2, fermionic)
    E = (0.41, -0.93)
    w = 1j * 2 * np.pi / beta
    got, terms = _oracle_value(alpha, eps, 2, fermionic, E, [w], beta)
    assert any(abs(code) == 2 for _, leaves, _ in terms for code, _ in leaves)
    ref = brute_force(alpha, eps, 2, E, [w], beta)
    assert abs(got - ref) <= 2e-6 * abs(ref), (got, ref)


@pytest.mark.parametrize("order,i", [(2, 0), (3, 1), (4, 1)])
def test_simple_poles_unchanged_by_the_option(order, i):
    d = random_self_energy(order, (0, order, i))
    a = canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))
    b = canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic, multipole=True))
    assert a == b
