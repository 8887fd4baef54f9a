"""Poles of higher order (Eq. (5)) on the GPU: the specialized forward kernels
with Taylor-coefficient leaves and groups of unequal denominator lists, on the
energy input, the momentum input and the in-kernel Monte-Carlo sums, against
the oracle's multipole solution; their adjoint, in one pass and in passes
over a workspace, against the oracle's analytic gradients (dT_j/dx =
(j + 1) T_(j+1)); the paths that do not take such solutions refuse them; the
batch takes them on the specialized kernels."""
import types

import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, real_freqs, uniform_energies
from oracle.evaluate import energies_from_k, gradients, momentum_gradients
from oracle.mc import draw_momenta

from parity import (NEAR, TOL, TOL_NEAR, check, far_from_poles, gradient_scales, reference,
                    reference_hubbard)
from multipole_cases import CASES, repeated_line
from test_multipole_cpu import _oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


def _diagram(case):
    alpha, eps, n_int, ferm = case
    return types.SimpleNamespace(alpha=alpha, eps=eps, n_int=n_int, fermionic=ferm)


def hubbard_case(order, i, line=0):
    """The repeated-line diagram in the momentum form: one energy per line, the
    repeated line's energy slot unused (both copies read the first one)."""
    alpha, eps, n_int, ferm = repeated_line(order, i, line)
    ng = alpha.shape[0]
    j = [r for r in range(ng - 1) if np.array_equal(alpha[r], alpha[-1])][0]
    e = np.eye(ng, dtype=np.int8)
    e[-1] = 0
    e[-1, j] = 1
    return alpha, e, n_int, ferm


@pytest.mark.parametrize("name", list(CASES))
def test_multipole_energy_path(name):
    case = CASES[name]
    d = _diagram(case)
    T = amd.Terms(*case, multipole=True)
    beta = 4.0
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -3.0, 3.0, 0.05)])
    if not case[3][-1]:
        w = np.concatenate([2j * np.pi * np.arange(1, 3) / beta, real_freqs(2, -3.0, 3.0, 0.05)])
    E = uniform_energies(1300, case[1].shape[1], seed=(45, d.n_int, case[0].shape[0]), a=3.0)
    Et = torch.from_numpy(E).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    out, s = amd.evaluate(T, Et, wt, beta, want_out=True, want_sum=True)
    torch.cuda.synchronize()
    assert amd.last_variant().startswith("specialized")
    terms = _oracle(case)
    ref, scale, dist = reference(d, E, w, beta, terms=terms)
    check(out.cpu().numpy(), ref, scale, dist, label=f"{name} multipole energies")
    far = (dist >= NEAR).all(axis=0)
    np.testing.assert_allclose(s.cpu().numpy(), out.cpu().numpy().sum(axis=1), rtol=1e-12,
                               atol=1e-12 * scale.sum())
    assert far.sum() > 1000


@pytest.mark.parametrize("order,i,line", [(3, 0, 0), (4, 1, 0), (4, 3, 1)])
def test_multipole_momentum_path_and_mc(order, i, line):
    case = hubbard_case(order, i, line)
    d = _diagram(case)
    terms = _oracle(case)
    T = amd.Terms(*case, multipole=True)
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(2, -4.0, 4.0, 0.05)])
    k = k_samples(1100, d.n_int, seed=(46, order, i))
    out, _ = amd.evaluate_hubbard(T, torch.from_numpy(k).to(DEV), q, t, mu, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta, terms=terms)
    check(out.cpu().numpy(), ref, scale, dist, label=f"order {order} multipole momenta")
    # Monte-Carlo sums with the momenta drawn in the kernel
    n, seed = 5000, 77
    sums = amd.integrate_hubbard(T, n, seed, q, t, mu, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    kd = draw_momenta(0, n, 2 * d.n_int, seed)
    ref, scale, dist, _ = reference_hubbard(d, kd, q, t, mu, w, beta, terms=terms)
    tol = np.where(dist >= NEAR, TOL, TOL_NEAR) * scale
    want = np.stack([ref.real.sum(1), ref.imag.sum(1), (ref.real ** 2).sum(1), (ref.imag ** 2).sum(1)], axis=1)
    bound = np.stack([tol.sum(1), tol.sum(1), (2 * np.abs(ref) * tol).sum(1), (2 * np.abs(ref) * tol).sum(1)],
                     axis=1)
    assert np.all(np.abs(sums.cpu().numpy() - want) <= bound + 1e-300)


def test_multipole_refusals():
    case = CASES["double"]
    T = amd.Terms(*case, multipole=True)
    T.specialize(momentum=False)           # forward and adjoint
    E = torch.from_numpy(uniform_energies(64, 2, seed=47, a=3.0)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(2, 2.0) * 2).to(DEV)
    for v in (amd.VARIANT_TABLES, amd.VARIANT_PACKED):
        T.set_variant(v)
        with pytest.raises(amd.AmiError) as e:
            amd.evaluate(T, E, w, 2.0)
        assert e.value.code == -7
        with pytest.raises(amd.AmiError) as e:
            amd.evaluate_adjoint(T, E, w, 2.0, grad_out=torch.ones((2, 64), dtype=torch.complex128, device=DEV))
        assert e.value.code == -7
    T.set_variant(amd.VARIANT_AUTO)
    out, _ = amd.evaluate(T, E, w, 2.0)
    # a batch takes the item on its specialized kernels (equal to the call
    # above bit for bit); the packed-only batch refuses it
    o = torch.empty((2, 64), dtype=torch.complex128, device=DEV)
    b = amd.Batch([{"terms": T, "energies": E, "ext_freqs": w, "beta": 2.0, "out": o}])
    b.run()
    torch.cuda.synchronize()
    assert b.info()["specialized_items"] == 1 and torch.equal(o, out)
    with pytest.raises(amd.AmiError) as e:
        amd.Batch([{"terms": T, "energies": E, "ext_freqs": w, "beta": 2.0, "out": o}], {"kernels": 1})
    assert e.value.code == -7


# the adjoint's specialized kernels: one pass, and passes over a workspace
ADJ = pytest.mark.parametrize("variant", [amd.VARIANT_SPECIALIZED, amd.VARIANT_TWO_PASS],
                              ids=["one_pass", "passes"])


@pytest.mark.parametrize("name", list(CASES))
@ADJ
def test_multipole_energy_adjoint(name, variant):
    """dL/dE, dL/dbeta and dL/dw of L = Re sum conj(c) I within 1e-10 of their
    rounding scales, and the values the adjoint returns on the way within the
    forward's bar, on samples away from poles."""
    case = CASES[name]
    d = _diagram(case)
    terms = _oracle(case)
    T = amd.Terms(*case, multipole=True)
    T.set_variant(variant)
    beta = 4.0
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.6, 0.6, 0.05)])
    if not case[3][-1]:
        w = np.concatenate([2j * np.pi * np.arange(1, 3) / beta, real_freqs(1, 0.6, 0.6, 0.05)])
    E = uniform_energies(700, case[1].shape[1], seed=(49, d.n_int, case[0].shape[0]), a=3.0)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    rng = np.random.default_rng(50)
    cot = rng.standard_normal((len(w), len(E))) + 1j * rng.standard_normal((len(w), len(E)))
    cot_sum = np.array([0.3 - 0.2j, -0.1j, 0.25])
    out = torch.empty((len(w), len(E)), dtype=torch.complex128, device=DEV)
    g_e, g_b, g_w = amd.evaluate_adjoint(T, torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), beta,
                                         grad_out=torch.from_numpy(cot).to(DEV),
                                         grad_sum=torch.from_numpy(cot_sum).to(DEV), out=out)
    torch.cuda.synchronize()
    assert amd.last_variant() == ("specialized" if variant == amd.VARIANT_SPECIALIZED else "specialized passes")
    full = cot + cot_sum[:, None]
    ref_e, ref_b, ref_w = gradients(terms, d.n_int, E, w, beta, full)
    sc = gradient_scales(terms, d.n_int, E, w, beta, full)
    assert np.max(np.abs(g_e.cpu().numpy() - ref_e.astype(np.float64)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(float(g_b) - float(ref_b)) <= 1e-10 * sc["beta"]
    if case[0].shape[1] > d.n_int:
        assert np.max(np.abs(g_w.cpu().numpy() - ref_w.astype(np.complex128))) <= 1e-10 * sc["w"]
    ref, scale, dist = reference(d, E, w, beta, terms=terms)
    check(out.cpu().numpy(), ref, scale, dist, label=f"{name} multipole adjoint values")


@pytest.mark.parametrize("order,i,line", [(3, 0, 0), (4, 1, 0)])
@ADJ
def test_multipole_momentum_adjoint(order, i, line, variant):
    """The momentum path's adjoint of a repeated-line diagram: dL/dk, dL/dmu,
    dL/dt, dL/dbeta and dL/dw within 1e-10 of their rounding scales."""
    case = hubbard_case(order, i, line)
    d = _diagram(case)
    terms = _oracle(case)
    T = amd.Terms(*case, multipole=True)
    T.set_variant(variant)
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    k = k_samples(600, d.n_int, seed=(51, order, i))
    k = np.ascontiguousarray(k[far_from_poles(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu), w)])
    rng = np.random.default_rng(52)
    cot = rng.standard_normal((1, len(k))) + 1j * rng.standard_normal((1, len(k)))
    g_k, g_mu, g_t, g_b, g_w = amd.evaluate_hubbard_adjoint(
        T, torch.from_numpy(k).to(DEV), q, t, mu, torch.from_numpy(w).to(DEV), beta,
        grad_out=torch.from_numpy(cot).to(DEV))
    torch.cuda.synchronize()
    E = energies_from_k(d.alpha, k, q, t, mu)
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, hubbard=(d.alpha, k, q, t, mu))
    assert np.max(np.abs(g_k.cpu().numpy() - dk.astype(np.float64)) / np.maximum(sc["k"], 1e-300)) <= 1e-10
    for got, want, key in ((g_b, db, "beta"), (g_mu, dmu, "mu"), (g_t, dt, "t")):
        assert abs(float(got) - float(want)) <= 1e-10 * sc[key], key
    assert np.max(np.abs(g_w.cpu().numpy() - dw.astype(np.complex128))) <= 1e-10 * sc["w"]
