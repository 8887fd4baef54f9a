"""Pins of the oracle at complex energies (the energy vector's element type is
complex, Sec. 5.1.3): the textbook second-order form continued to complex
energies, the plain definition Eq. (1) by truncated Matsubara sums, the
Cauchy-Riemann relations of an analytic function of the energies, conjugation
symmetry, the real limit, leaves far out on both sides, and the analytic
gradients at complex energies against central differences of the values in
the real and the imaginary direction of every energy (CPU only)."""
import numpy as np
import pytest

from ami_inputs import complex_energies, matsubara_freqs, order2_example, random_self_energy, uniform_energies
from oracle.brute import brute_force
from oracle.construct import canonical, construct
from oracle.evaluate import CLD, LD, evaluate_terms, gradients, leaf_value, term_magnitudes


def _terms(d, multipole=False):
    return canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic, multipole=multipole))


def test_order2_textbook_form_at_complex_energies():
    """-[f1 f3 (1-f2) + (1-f1)(1-f3) f2] / (i nu + xi2 - xi1 - xi3), xi = -E,
    with f(xi) = 1/(exp(beta xi) + 1) taken at complex xi."""
    d = order2_example()
    beta = 5.0
    E = complex_energies(150, 3, seed=81)
    w = matsubara_freqs(3, beta)
    got = evaluate_terms(_terms(d), 2, E, w, beta).astype(np.complex128)
    xi = -E
    f1, f2, f3 = (1.0 / (np.exp(beta * xi[:, i]) + 1.0) for i in range(3))
    num = f1 * f3 * (1 - f2) + (1 - f1) * (1 - f3) * f2
    for j in range(3):
        want = -num / (w[j] + xi[:, 1] - xi[:, 0] - xi[:, 2])
        np.testing.assert_allclose(got[j], want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("E", [(0.7 + 0.2j, -1.3 - 0.05j), (-0.4 - 0.3j, 0.9 + 0.1j)])
def test_bubble_against_brute_force_at_complex_energies(E):
    alpha = np.array([[1, 0], [1, 1]])
    eps = np.eye(2, dtype=int)
    beta = 2.0
    terms = canonical(construct(alpha, eps, 1, fermionic=[1, 0]))
    for Om in (2 * np.pi / beta, 4 * np.pi / beta):
        got = complex(evaluate_terms(terms, 1, np.array([E]), np.array([1j * Om]), beta)[0, 0])
        ref = brute_force(alpha, eps, 1, np.array(E), [1j * Om], beta)
        assert abs(got - ref) <= 1e-9 * abs(ref), (got, ref)


def test_order2_and_double_pole_against_brute_force_at_complex_energies():
    d = order2_example()
    beta = 3.0
    E = np.array([0.37 + 0.11j, -1.21 - 0.07j, 0.83 + 0.04j])
    w = 1j * np.pi / beta
    got = complex(evaluate_terms(_terms(d), 2, E[None, :], np.array([w]), beta)[0, 0])
    ref = brute_force(d.alpha, d.eps, 2, E, [w], beta)
    assert abs(got - ref) <= 1e-6 * abs(ref), (got, ref)
    # a double pole (Eq. (5)) at complex energies
    alpha = np.array([[1, 0], [1, 0], [1, 1]])
    eps = np.array([[1, 0], [1, 0], [0, 1]])
    terms = canonical(construct(alpha, eps, 1, [1, 0], multipole=True))
    E2 = np.array([0.45 - 0.2j, -0.8 + 0.15j])
    for Om in (2 * np.pi / beta, 4 * np.pi / beta):
        got = complex(evaluate_terms(terms, 1, E2[None, :], np.array([1j * Om]), beta)[0, 0])
        ref = brute_force(alpha, eps, 1, E2, [1j * Om], beta)
        assert abs(got - ref) <= 1e-8 * abs(ref), (got, ref)


@pytest.mark.parametrize("order,i", [(3, 0), (4, 1)])
def test_cauchy_riemann_in_every_energy(order, i):
    """An analytic function of E_j changes along i e_j by i times its change
    along e_j: central differences of the two agree to their truncation
    error.  A conjugate taken where it should not be, or a leaf continued
    in the wrong variable, breaks this."""
    d = random_self_energy(order, (0, order, i))
    terms = _terms(d)
    beta = 2.0
    E0 = complex_energies(6, d.n_eps, seed=(82, order), eta=0.05).astype(CLD)
    w = matsubara_freqs(1, beta)
    h = LD(1e-5)
    for j in range(d.n_eps):
        ej = np.zeros(d.n_eps, dtype=CLD)
        ej[j] = 1
        dre = (evaluate_terms(terms, d.n_int, E0 + h * ej, w, beta)
               - evaluate_terms(terms, d.n_int, E0 - h * ej, w, beta)) / (2 * h)
        dim = (evaluate_terms(terms, d.n_int, E0 + 1j * h * ej, w, beta)
               - evaluate_terms(terms, d.n_int, E0 - 1j * h * ej, w, beta)) / (2 * h)
        scale = np.max(np.abs(dre)) + 1e-300
        assert np.max(np.abs(dim - 1j * dre)) <= 1e-6 * scale, j


def test_conjugation_and_real_limit():
    d = random_self_energy(4, (0, 4, 3))
    terms = _terms(d)
    beta = 4.0
    E = complex_energies(100, d.n_eps, seed=83)
    w = np.concatenate([matsubara_freqs(2, beta), [0.3 + 0.05j]])
    a = evaluate_terms(terms, d.n_int, E, w, beta)
    b = evaluate_terms(terms, d.n_int, np.conj(E), np.conj(w), beta)
    np.testing.assert_allclose(b.astype(np.complex128), np.conj(a).astype(np.complex128), rtol=1e-15)
    Er = uniform_energies(100, d.n_eps, seed=84, a=3.0)
    real = evaluate_terms(terms, d.n_int, Er, w, beta)
    cplx = evaluate_terms(terms, d.n_int, Er.astype(np.complex128), w, beta)
    scale = term_magnitudes(terms, d.n_int, Er, w, beta).astype(np.float64) + 1e-300
    assert np.max(np.abs((cplx - real).astype(np.complex128)) / scale) <= 1e-17


@pytest.mark.parametrize("sigma", [1, -1])
def test_complex_leaves_far_out(sigma):
    """No overflow on either side: both kinds of leaf tend to 0 as Re y -> +inf
    and to 1 as Re y -> -inf (1/(e^y + 1) and 1/(1 - e^y))."""
    y = np.array([2000 + 1j, -2000 + 3j, 40 - 2j, -40 + 0.5j], dtype=CLD)
    f = leaf_value(sigma, y)
    assert np.all(np.isfinite(f.real)) and np.all(np.isfinite(f.imag))
    assert abs(f[0]) < 1e-300 and abs(f[1] - 1) < 1e-18
    # at moderate arguments the leaf equals the plain formula
    np.testing.assert_allclose(f[2:].astype(np.complex128),
                               (1 / (sigma * np.exp(y[2:]) + 1)).astype(np.complex128), rtol=1e-15)


@pytest.mark.parametrize("order,i,e_reg", [(2, None, 0.0), (3, 0, 0.0), (4, 1, 0.0), (4, 3, 0.02)])
def test_complex_gradients_against_central_differences(order, i, e_reg):
    """dL/dRe E_j + i dL/dIm E_j of L = Re sum conj(c) I at complex energies,
    dL/dbeta and dL/dw, against long-double central differences of the
    oracle's values (step 1e-6: truncation and rounding below 1e-9 of each
    gradient's scale); at real energies the real part is the real-energy
    gradient.  A missing conjugate, a sign of the imaginary direction or a
    leaf slope continued wrongly fails one of them."""
    from parity import gradient_scales
    d = order2_example() if i is None else random_self_energy(order, (0, order, i))
    terms = _terms(d)
    beta = 2.0
    E = complex_energies(4, d.n_eps, seed=(85, order), eta=0.1).astype(CLD)
    w = np.concatenate([matsubara_freqs(1, beta), [0.4 + 0.06j]])[:, None].astype(CLD)
    rng = np.random.default_rng(86)
    cot = rng.standard_normal((2, 4)) + 1j * rng.standard_normal((2, 4))

    def loss(Ev, b, wv=w):
        v = evaluate_terms(terms, d.n_int, Ev, wv, b, e_reg)
        return np.real(np.sum(np.conj(cot) * v, axis=0))            # per sample

    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot, e_reg, per_sample=True)
    assert np.iscomplexobj(dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, e_reg)
    h = LD(1e-6)
    for j in range(d.n_eps):
        ej = np.zeros(d.n_eps, dtype=CLD)
        ej[j] = 1
        fre = (loss(E + h * ej, beta) - loss(E - h * ej, beta)) / (2 * h)
        fim = (loss(E + 1j * h * ej, beta) - loss(E - 1j * h * ej, beta)) / (2 * h)
        err = np.abs(dE[:, j] - (fre + 1j * fim))
        assert np.all(err <= 1e-9 * np.maximum(sc["E"][:, j], 1e-300)), (j, dE[:, j], fre + 1j * fim)
    fb = (loss(E, LD(beta) + h) - loss(E, LD(beta) - h)) / (2 * h)
    assert abs(float(np.sum(db)) - float(np.sum(fb))) <= 1e-9 * sc["beta"]
    for f in range(2):
        df = np.zeros_like(w)
        df[f, 0] = 1
        fre = np.sum(loss(E, beta, w + h * df) - loss(E, beta, w - h * df)) / (2 * h)
        fim = np.sum(loss(E, beta, w + 1j * h * df) - loss(E, beta, w - 1j * h * df)) / (2 * h)
        assert abs(complex(np.sum(dw[f, :, 0])) - complex(fre + 1j * fim)) <= 1e-9 * sc["w"], f
    # the real limit: real energies given as complex numbers
    Er = uniform_energies(5, d.n_eps, seed=87, a=3.0)
    c5 = rng.standard_normal((2, 5)) + 1j * rng.standard_normal((2, 5))
    gr, br, wr = gradients(terms, d.n_int, Er, w, beta, c5, e_reg)
    gc, bc, wc = gradients(terms, d.n_int, Er.astype(np.complex128), w, beta, c5, e_reg)
    scr = gradient_scales(terms, d.n_int, Er, w, beta, c5, e_reg)
    assert np.max(np.abs(np.real(gc) - gr) / np.maximum(scr["E"], 1e-300)) <= 1e-17
    assert abs(float(bc) - float(br)) <= 1e-17 * scr["beta"]
    assert np.max(np.abs(wc - wr)) <= 1e-17 * scr["w"]
