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

from multipole_cases import CASES, SINGLE_SUM_CASES


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


def _residue_sum_mpmath(alpha, eps, E, w, beta):
    """The residue theorem for one sum written out directly: the poles of
    prod_j 1/(a_j z + c_j) (z = i nu), each of order M, contribute
    (1/(M-1)!) d^(M-1)/dz^(M-1) [f(beta z) (z - z0)^M prod_j 1/(a_j z + c_j)]
    at z0, with f(y) = 1/(exp(y) + 1) taken at the complex pole itself (no
    periodicity argument) and the derivative by 40-digit numerical
    differentiation."""
    mp.mp.dps = 40
    a = [int(r[0]) for r in alpha]
    c = [sum(int(eps[j][i]) * mp.mpf(E[i]) for i in range(len(E))) + int(alpha[j][1]) * mp.mpc(w)
         for j in range(len(a))]
    poles = {}
    for j in range(len(a)):
        z0 = -c[j] / a[j]
        key = (mp.nstr(mp.re(z0), 25), mp.nstr(mp.im(z0), 25))
        poles.setdefault(key, (z0, []))[1].append(j)
    total = mp.mpc(0)
    for z0, members in poles.values():
        M = len(members)
        rest = [j for j in range(len(a)) if j not in members]

        def h(z, members=members, rest=rest):
            v = 1 / (mp.exp(beta * z) + 1)
            for j in members:
                v /= a[j]            # (z - z0) / (a_j z + c_j) = 1 / a_j
            for j in rest:
                v /= a[j] * z + c[j]
            return v
        total += mp.diff(h, z0, M - 1) / mp.factorial(M - 1)
    return complex(total)


@pytest.mark.parametrize("name", list(SINGLE_SUM_CASES))
def test_higher_order_single_sums(name):
    import oracle.construct as oc
    alpha, eps, n_int, fermionic = SINGLE_SUM_CASES[name]
    beta = 2.0
    with pytest.raises(MultipoleError):
        construct(alpha, eps, 1, fermionic)
    # record which Leibniz factors (m, k) the construction takes
    seen = set()
    binom = oc._binom

    def spy(n, k):
        seen.add((n - k + 1, k))
        return binom(n, k)
    oc._binom = spy
    try:
        terms = canonical(construct(alpha, eps, n_int, fermionic, multipole=True))
    finally:
        oc._binom = binom
    want_codes = {"triple": 3, "quadruple": 4, "square_square": 2, "square_negsquare": 2, "triple_square": 3}[name]
    assert max(abs(code) for _, leaves, _ in terms for code, _ in leaves) == want_codes
    if name != "triple" and name != "quadruple":
        assert any(m >= 2 and k >= 1 for m, k in seen), seen
    for E, Om in (((0.37, -1.21), 2 * np.pi / beta), ((-0.8, 0.45), 4 * np.pi / beta)):
        w = 1j * Om
        got = complex(evaluate_terms(terms, n_int, np.array([E]), np.array([[w]]), beta)[0, 0])
        ref = brute_force(alpha, eps, 1, E, [w], beta)
        assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)
        res = _residue_sum_mpmath(alpha, eps, E, w, beta)
        assert abs(got - res) <= 1e-13 * abs(res), (got, res)


def test_double_poles_at_three_sums_against_brute_force():
    """The order-3 self-energy with one line taken twice (a constant
    self-energy inserted on it): double poles over three nested sums, against
    the truncated triple sum of Eq. (1)."""
    alpha, eps, n_int, ferm = CASES["o3"]
    assert n_int == 3
    beta = 2.0
    terms = canonical(construct(alpha, eps, n_int, ferm, multipole=True))
    assert any(abs(code) == 2 for _, leaves, _ in terms for code, _ in leaves)
    for E in ((0.41, -0.93, 0.77, -0.35, 1.12), (-0.62, 0.31, -1.37, 0.93, 0.19)):
        w = 1j * np.pi / beta
        got = complex(evaluate_terms(terms, n_int, np.array([E]), np.array([[w]]), beta)[0, 0])
        ref = brute_force(alpha, eps, n_int, E, [w], beta)
        assert abs(got - ref) <= 3e-6 * abs(ref), (got, ref)


def test_double_pole_values_invariant_under_relabelling():
    """Reordering and negating the summed frequencies of the order-4 solution
    with a repeated line changes its term list, not its value."""
    from oracle.construct import CoeffError
    alpha, eps, n_int, ferm = CASES["o4"]
    beta = 3.0
    E = np.array([[0.41, -0.93, 0.77, -0.35, 1.12, -0.58, 0.26][:eps.shape[1]],
                  [-0.3, 0.65, -1.1, 0.2, 0.85, 0.44, -0.71][:eps.shape[1]]])
    w = np.array([[1j * np.pi / beta], [0.4 + 0.05j]])
    base = evaluate_terms(canonical(construct(alpha, eps, n_int, ferm, multipole=True)), n_int, E, w, beta)
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(12):
        perm = list(rng.permutation(n_int))
        signs = list(rng.choice([-1, 1], size=n_int))
        cols = perm + list(range(n_int, alpha.shape[1]))
        a2 = alpha[:, cols].astype(np.int64)
        a2[:, :n_int] *= np.asarray(signs)[None, :]
        rows = list(reversed(range(alpha.shape[0])))
        try:
            t2 = canonical(construct(a2[rows], eps[rows], n_int, [ferm[c] for c in cols], multipole=True))
        except CoeffError:
            continue
        other = evaluate_terms(t2, n_int, E, w, beta)
        np.testing.assert_allclose(other.astype(np.complex128), base.astype(np.complex128), rtol=1e-11, atol=1e-14)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("sigma", [1, -1])
@pytest.mark.parametrize("j", [0, 1, 2])
def test_taylor_leaf_slopes_against_mpmath(sigma, j):
    """The derivatives the gradients take of a Taylor-coefficient leaf:
    dT_j/dx = (j + 1) T_(j+1) and dT_j/dbeta = (j T_j + x (j + 1) T_(j+1)) / beta,
    against 40-digit differentiation of T_j(x; beta) = (1/j!) d^j/dx^j f(beta x)."""
    mp.mp.dps = 40

    def T(x, b):
        return mp.diff(lambda u: 1 / (sigma * mp.exp(b * u) + 1), x, j) / mp.factorial(j)
    for x, beta in ((-1.3, 2.5), (0.42, 2.5), (2.2, 1.3)):
        X, B = mp.mpf(x), mp.mpf(beta)
        want_x = mp.diff(lambda u: T(u, B), X)
        want_b = mp.diff(lambda b: T(X, b), B)
        lx, lb = np.longdouble(x), np.longdouble(beta)
        tj = leaf_coefficient(sigma * (j + 1), lx, lb)
        slope = (j + 1) * leaf_coefficient(sigma * (j + 2), lx, lb)
        got_b = (j * tj + lx * slope) / lb
        assert abs(float(slope) - float(want_x)) <= 1e-14 * abs(float(want_x)) + 1e-300
        assert abs(float(got_b) - float(want_b)) <= 1e-14 * abs(float(want_b)) + 1e-300


@pytest.mark.parametrize("name", ["double", "later", "o3", "o4", "triple", "square_square", "triple_square"])
def test_multipole_gradients_against_finite_differences(name):
    """The oracle's analytic gradients of solutions with poles of higher order
    (Taylor-coefficient leaves, powers of denominators) against central
    differences of its own long-double values (step 1e-6: truncation and
    rounding both below 1e-10 of the gradient's scale)."""
    from oracle.evaluate import gradients
    from parity import gradient_scales
    alpha, eps, n_int, ferm = (CASES if name in CASES else SINGLE_SUM_CASES)[name]
    terms = canonical(construct(alpha, eps, n_int, ferm, multipole=True))
    assert any(abs(code) > 1 for _, leaves, _ in terms for code, _ in leaves)
    beta = 2.0
    rng = np.random.default_rng(11)
    E = rng.uniform(-1.5, 1.5, size=(3, eps.shape[1])).astype(np.longdouble)
    n_ext = alpha.shape[1] - n_int
    w = np.array([[1j * np.pi / beta] * n_ext, [0.35 + 0.05j] * n_ext]) if n_ext else np.zeros((2, 0))
    if name in SINGLE_SUM_CASES:     # bosonic external: an even Matsubara frequency
        w = np.array([[2j * np.pi / beta] * n_ext, [0.35 + 0.05j] * n_ext])
    cot = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))

    def loss(Ev, b):
        v = evaluate_terms(terms, n_int, Ev, w, b)
        return np.real(np.sum(np.conj(cot) * v, axis=0))            # per sample
    dE, db, _ = gradients(terms, n_int, E, w, beta, cot, per_sample=True)
    sc = gradient_scales(terms, n_int, E, w, beta, cot)
    h = np.longdouble(1e-6)
    for i in range(E.shape[1]):
        ep, em = E.copy(), E.copy()
        ep[:, i] += h
        em[:, i] -= h
        fd = (loss(ep, beta) - loss(em, beta)) / (2 * h)
        assert np.all(np.abs(dE[:, i] - fd) <= 1e-9 * np.maximum(sc["E"][:, i], 1e-300)), (i, dE[:, i], fd)
    fd_b = (loss(E, np.longdouble(beta) + h) - loss(E, np.longdouble(beta) - h)) / (2 * h)
    assert abs(float(np.sum(db)) - float(np.sum(fd_b))) <= 1e-9 * sc["beta"]
