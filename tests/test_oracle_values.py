"""Pins of the oracle's values: closed forms, brute-force Matsubara sums of
Eq. (1), invariants, the printed momentum mapping, gradients (CPU only)."""
import os

import numpy as np
import pytest

from ami_inputs import (k_samples, matsubara_freqs, order2_example,
                        random_self_energy, real_freqs, relabel,
                        uniform_energies)
from oracle.brute import brute_force
from oracle.construct import (CoeffError, canonical, construct, construct_tree)
from oracle.evaluate import (LD, energies_from_k, evaluate_terms, evaluate_tree,
                             gradients, kron_alpha, line_momenta,
                             momentum_gradients)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _terms(d):
    return canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))


def _fermi(beta, x):
    return 1.0 / (np.exp(beta * x) + 1.0)


def test_order2_textbook_closed_form():
    """Second-order self-energy in the usual textbook form, with xi = -E:
    -[f1 f3 (1-f2) + (1-f1)(1-f3) f2] / (i nu + xi2 - xi1 - xi3)."""
    d = order2_example()
    terms = _terms(d)
    beta = 5.0
    E = uniform_energies(200, 3, seed=11, a=4.0)
    w = matsubara_freqs(3, beta)
    got = evaluate_terms(terms, 2, E, w, beta)
    xi = -E
    f1, f2, f3 = (_fermi(beta, xi[:, i]) for i in range(3))
    num = f1 * f3 * (1 - f2) + (1 - f1) * (1 - f3) * f2
    for j in range(3):
        want = -num / (w[j] + xi[:, 1] - xi[:, 0] - xi[:, 2])
        np.testing.assert_allclose(got[j].astype(np.complex128), want, rtol=1e-13, atol=1e-15)


def test_single_sum_closed_form():
    """(1/beta) sum_nu 1/((i nu + E1)(i nu + i Omega + E2)) with a bosonic
    Omega equals [f(-E1) - f(-E2)] / (i Omega + E2 - E1)."""
    alpha = np.array([[1, 0], [1, 1]])
    eps = np.eye(2, dtype=int)
    terms = canonical(construct(alpha, eps, 1, fermionic=[1, 0]))
    beta = 2.5
    E = uniform_energies(50, 2, seed=3, a=3.0)
    W = 1j * 2 * np.pi * np.arange(0, 4) / beta
    got = evaluate_terms(terms, 1, E, W, beta)
    for j, Om in enumerate(W):
        want = (_fermi(beta, -E[:, 0]) - _fermi(beta, -E[:, 1])) / (Om + E[:, 1] - E[:, 0])
        np.testing.assert_allclose(got[j].astype(np.complex128), want, rtol=1e-12)


def test_brute_force_single_sums():
    beta = 3.0
    cases = [
        (np.array([[1, 0], [1, 1]]), [1, 0], 2j * np.pi / beta),
        (np.array([[1, 0], [-1, 1]]), [1, 1], 1j * np.pi / beta),
        (np.array([[1, 0], [1, 1], [-1, 1]]), [1, 0], 4j * np.pi / beta),
    ]
    rng = np.random.default_rng(4)
    for alpha, ferm, w in cases:
        eps = np.eye(alpha.shape[0], dtype=int)
        E = rng.uniform(-2, 2, alpha.shape[0])
        terms = canonical(construct(alpha, eps, 1, fermionic=ferm))
        ref = complex(evaluate_terms(terms, 1, E[None], np.array([w]), beta)[0, 0])
        bf = brute_force(alpha, eps, 1, E, np.array([w]), beta)
        assert abs(bf - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("which", ["paper", 0, 1, 2])
def test_brute_force_order2(which):
    d = order2_example() if which == "paper" else random_self_energy(2, (0, 2, which))
    terms = _terms(d)
    beta = 5.0 if which == "paper" else 3.0
    rng = np.random.default_rng(7 + (0 if which == "paper" else which))
    E = rng.uniform(-2, 2, d.n_eps)
    if which == "paper":
        E = np.array([0.37, -1.21, 0.83])   # a point where the value is O(1)
    w = np.array([1j * np.pi / beta])
    ref = complex(evaluate_terms(terms, 2, E[None], w, beta)[0, 0])
    bf = brute_force(d.alpha, d.eps, 2, E, w, beta)
    assert abs(bf - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("i", [0, 2])
def test_brute_force_order3(i):
    d = random_self_energy(3, (0, 3, i))
    terms = _terms(d)
    beta = 3.0
    rng = np.random.default_rng(100 + i)
    E = rng.uniform(-2, 2, d.n_eps)
    w = np.array([1j * np.pi / beta])
    ref = complex(evaluate_terms(terms, 3, E[None], w, beta)[0, 0])
    bf = brute_force(d.alpha, d.eps, 3, E, w, beta)
    assert abs(bf - ref) <= 3e-5 * abs(ref)


@pytest.mark.parametrize("order", [3, 4])
def test_sign_flip_and_conjugation(order):
    """Eq. (1) with every energy and frequency negated is (-1)^nG times the
    original (the fermionic sums are symmetric); with real energies the
    conjugate frequency gives the conjugate value."""
    for i in range(3):
        d = random_self_energy(order, (2, order, i))
        terms = _terms(d)
        beta = 4.0
        E = uniform_energies(64, d.n_eps, seed=(5, i), a=3.0)
        w = matsubara_freqs(2, beta)
        a = evaluate_terms(terms, order, E, w, beta)
        b = evaluate_terms(terms, order, -E, -w, beta)
        c = evaluate_terms(terms, order, E, np.conj(w), beta)
        sgn = (-1) ** d.n_g
        np.testing.assert_allclose(b.astype(np.complex128), sgn * a.astype(np.complex128),
                                   rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(c.astype(np.complex128), np.conj(a.astype(np.complex128)),
                                   rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("order", [3, 4])
def test_summation_order_invariance(order):
    """Doing the sums in another order, or negating a summed frequency,
    changes the term list but not the value."""
    checked = 0
    for i in range(4):
        d = random_self_energy(order, (3, order, i))
        E = uniform_energies(32, d.n_eps, seed=(6, i), a=3.0)
        beta = 2.0
        w = matsubara_freqs(2, beta)
        ref = evaluate_terms(_terms(d), order, E, w, beta)
        perm = list(np.random.default_rng(i).permutation(order))
        signs = [1 if k % 2 else -1 for k in range(order)]
        r = relabel(d, perm, row_perm=list(reversed(range(d.n_g))), loop_sign=signs)
        try:
            other = evaluate_terms(_terms(r), order, E, w, beta)
        except CoeffError:
            continue
        np.testing.assert_allclose(other.astype(np.complex128), ref.astype(np.complex128),
                                   rtol=1e-11, atol=1e-13)
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("order,i", [(2, 0), (3, 1), (4, 2), (5, 3)])
def test_factorized_equals_flat_values(order, i):
    d = random_self_energy(order, (4, order, i))
    E = uniform_energies(40, d.n_eps, seed=(8, i), a=3.0)
    beta = 5.0
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -2, 2, 0.05)])
    flat = evaluate_terms(_terms(d), order, E, w, beta)
    tree = evaluate_tree(construct_tree(d.alpha, d.eps, d.n_int), order, E, w, beta)
    np.testing.assert_allclose(tree.astype(np.complex128), flat.astype(np.complex128),
                               rtol=1e-12, atol=1e-13)


def test_removable_bose_pole_is_finite():
    """At -E1-E3 -> 0 the Bose-type leaf of the order-2 solution diverges,
    but the total (Eq. (1) is regular there) stays continuous."""
    d = order2_example()
    terms = _terms(d)
    beta = 5.0
    w = matsubara_freqs(1, beta)
    vals = []
    for delta in (1e-6, -1e-6, 1e-9, -1e-9):
        E = np.array([[0.3, -0.4, -0.3 + delta]])
        per_term = [abs(complex(evaluate_terms([t], 2, E, w, beta)[0, 0])) for t in terms]
        total = complex(evaluate_terms(terms, 2, E, w, beta)[0, 0])
        assert max(per_term) > 1e4 * abs(total)
        vals.append(total)
    assert abs(vals[0] - vals[1]) < 1e-5 * abs(vals[0])
    assert abs(vals[2] - vals[3]) < 1e-8 * abs(vals[2])


def _read_matrix_blocks(path):
    blocks, name = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.isalpha():
            name = line
            blocks[name] = []
        else:
            blocks[name].append([int(x) for x in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_momentum_mapping_matches_printed_matrices():
    g = _read_matrix_blocks(os.path.join(GOLDEN, "kron_order2.txt"))
    d = order2_example()
    A = kron_alpha(d.alpha, 2)
    np.testing.assert_array_equal(A, g["A"])
    np.testing.assert_array_equal(A.T, g["AT"])
    k = k_samples(5, 2, seed=1)
    q = np.array([0.3, -0.2])
    K = line_momenta(d.alpha, k, q, 2)
    # K = (k1, k2, -k1 + k2 + q) per component (Sec. 5.2)
    want = np.concatenate([k[:, 0:2], k[:, 2:4], -k[:, 0:2] + k[:, 2:4] + q[None]], axis=1)
    np.testing.assert_allclose(K.astype(np.float64), want, rtol=0, atol=1e-15)


def test_hubbard_energies():
    d = order2_example()
    k = k_samples(7, 2, seed=2)
    q = np.array([np.pi / 2, np.pi / 2])
    E = energies_from_k(d.alpha, k, q, t=1.0, mu=0.3)
    k3 = -k[:, 0:2] + k[:, 2:4] + q
    want3 = 2 * (np.cos(k3[:, 0]) + np.cos(k3[:, 1])) + 0.3
    np.testing.assert_allclose(E[:, 2].astype(np.float64), want3, rtol=1e-14)
    want1 = 2 * (np.cos(k[:, 0]) + np.cos(k[:, 1])) + 0.3
    np.testing.assert_allclose(E[:, 0].astype(np.float64), want1, rtol=1e-14)


def test_float64_mode_agrees_with_longdouble():
    d = random_self_energy(4, (0, 4, 1))
    terms = _terms(d)
    E = uniform_energies(100, d.n_eps, seed=9, a=4.0)
    w = matsubara_freqs(1, 5.0)
    a = evaluate_terms(terms, 4, E, w, 5.0)
    b = evaluate_terms(terms, 4, E, w, 5.0, dtype=np.float64)
    np.testing.assert_allclose(b, a.astype(np.complex128), rtol=1e-10, atol=1e-12)


def _loss(terms, n, E, w, beta, cot):
    v = evaluate_terms(terms, n, E, w, beta)
    return float(np.sum(np.real(np.conj(cot) * v)))


def test_gradients_match_finite_differences():
    d = random_self_energy(3, (0, 3, 1))
    terms = _terms(d)
    beta = 4.0
    E = uniform_energies(3, d.n_eps, seed=12, a=2.0).astype(LD)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    rng = np.random.default_rng(0)
    cot = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    dE, db, dw = gradients(terms, 3, E, w, beta, cot)
    h = LD(1e-6)
    for s in range(3):
        for i in range(d.n_eps):
            Ep, Em = E.copy(), E.copy()
            Ep[s, i] += h
            Em[s, i] -= h
            fd = (_loss(terms, 3, Ep, w, beta, cot) - _loss(terms, 3, Em, w, beta, cot)) / (2 * h)
            assert abs(float(dE[s, i]) - fd) <= 1e-8 * max(1.0, abs(fd))
    fd = (_loss(terms, 3, E, w, beta + h, cot) - _loss(terms, 3, E, w, beta - h, cot)) / (2 * h)
    assert abs(float(db) - fd) <= 1e-8 * max(1.0, abs(fd))
    # complex frequency: d/d(Re w) of L equals Re(dw), d/d(Im w) equals Im(dw)
    for f in range(2):
        for comp, unit in ((np.real, 1.0), (np.imag, 1j)):
            wp, wm = w.astype(np.clongdouble), w.astype(np.clongdouble)
            wp[f] += unit * h
            wm[f] -= unit * h
            fd = (_loss(terms, 3, E, wp, beta, cot) - _loss(terms, 3, E, wm, beta, cot)) / (2 * h)
            assert abs(float(comp(dw[f, 0])) - fd) <= 1e-8 * max(1.0, abs(fd))


def test_momentum_gradients_match_finite_differences():
    d = order2_example()
    terms = _terms(d)
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array([np.pi / 2, np.pi / 2])
    k = k_samples(2, 2, seed=3).astype(LD)
    w = matsubara_freqs(1, beta)
    cot = np.array([[1.0 + 0.5j, -0.3 + 0.2j]])

    def loss(kk, m, tt=t):
        E = energies_from_k(d.alpha, kk, q, tt, m)
        return _loss(terms, 2, E, w, beta, cot)

    E = energies_from_k(d.alpha, k, q, t, mu)
    dE, _, _ = gradients(terms, 2, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    h = LD(1e-6)
    for s in range(2):
        for c in range(4):
            kp, km = k.copy(), k.copy()
            kp[s, c] += h
            km[s, c] -= h
            fd = (loss(kp, mu) - loss(km, mu)) / (2 * h)
            assert abs(float(dk[s, c]) - fd) <= 1e-8 * max(1.0, abs(fd))
    fd = (loss(k, mu + h) - loss(k, mu - h)) / (2 * h)
    assert abs(float(dmu) - fd) <= 1e-8 * max(1.0, abs(fd))
    fd = (loss(k, mu, t + h) - loss(k, mu, t - h)) / (2 * h)
    assert abs(float(dt) - fd) <= 1e-8 * max(1.0, abs(fd))
