"""Complex energies on the GPU (amiEvaluateComplex, the specialized
complex-energy kernel) against the oracle, element by element on seeded
inputs: sizes with ragged blocks, Matsubara and real frequencies, strided
energies, the regulator, row sums, the real limit against amiEvaluate, and
the refusals; the two-pass complex forward (solutions above 1024 terms, or
forced) with several chunks; the adjoint at complex energies (amiEvaluateComplexAdjoint)
against the oracle's analytic gradients, in the real limit against
amiEvaluateAdjoint, and its refusals."""
import numpy as np
import pytest

from ami_inputs import (complex_energies, matsubara_freqs, order2_example, random_self_energy, real_freqs,
                        uniform_energies)

from oracle.evaluate import gradients

from parity import check, far_from_poles, gradient_scales, oracle_terms, reference

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


def _diag(order, i):
    return order2_example() if i is None else random_self_energy(order, (0, order, i))


@pytest.mark.parametrize("order,i,beta,n_e,e_reg", [
    (2, None, 5.0, 1000, 0.0), (3, 0, 2.0, 1500, 0.0), (4, 1, 5.0, 2049, 0.0), (4, 6, 2.0, 777, 0.3),
    (5, 2, 5.0, 700, 0.0), (6, 0, 5.0, 300, 0.0),
])
def test_complex_energy_parity(order, i, beta, n_e, e_reg):
    d = _diag(order, i)
    # |beta Im x| stays below pi/2 for every leaf (no Fermi pole nearby)
    eta = 0.25 / (beta * d.n_int)
    E = complex_energies(n_e, d.n_eps, seed=(91, order, i or 0), a=3.0, eta=eta)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -4.0, 4.0, 0.05)])
    T = amd.Terms.from_diagram(d)
    out, s = amd.evaluate_complex(T, torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), beta, e_reg,
                                  want_out=True, want_sum=True)
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized complex"
    ref, scale, dist = reference(d, E, w, beta, e_reg)
    got = out.cpu().numpy()
    check(got, ref, scale, dist, label=f"complex order {order}")
    np.testing.assert_allclose(s.cpu().numpy(), got.sum(axis=1), rtol=1e-12, atol=1e-12 * scale.sum())


def test_complex_strided_bosonic_and_empty():
    # the bubble with a bosonic external frequency, energies read from a strided view
    alpha = np.array([[1, 0], [1, 1]])
    T = amd.Terms(alpha, np.eye(2, dtype=np.int8), 1, [1, 0])
    beta = 2.0
    big = complex_energies(613, 5, seed=92, a=3.0, eta=0.2)
    Et = torch.from_numpy(big).to(DEV)[:, 1:3]
    assert Et.stride() == (5, 1)
    w = 2j * np.pi * np.arange(1, 4) / beta
    out, _ = amd.evaluate_complex(T, Et, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    E = big[:, 1:3]
    f = lambda z: 1.0 / (np.exp(beta * z) + 1.0)
    closed = (f(-E[:, 0]) - f(-E[:, 1]))[None, :] / (w[:, None] + E[None, :, 1] - E[None, :, 0])
    np.testing.assert_allclose(out.cpu().numpy(), closed, rtol=1e-12, atol=1e-14)
    # the transposed layout (stride_i > stride_s)
    Tt = torch.from_numpy(np.ascontiguousarray(E.T)).to(DEV).t()
    out2, _ = amd.evaluate_complex(T, Tt, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    assert torch.equal(out2, out)
    # no samples: zero row sums
    _, s0 = amd.evaluate_complex(T, Et[:0], torch.from_numpy(w).to(DEV), beta, want_out=False, want_sum=True)
    torch.cuda.synchronize()
    assert torch.all(s0 == 0)


def test_complex_real_limit_matches_the_real_path():
    d = random_self_energy(4, (0, 4, 3))
    T = amd.Terms.from_diagram(d)
    beta = 5.0
    E = uniform_energies(1024, d.n_eps, seed=93, a=3.0)
    w = torch.from_numpy(np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.5, 0.5, 0.05)])).to(DEV)
    Er = torch.from_numpy(E).to(DEV)
    a, _ = amd.evaluate(T, Er, w, beta)
    b, _ = amd.evaluate_complex(T, Er.to(torch.complex128), w, beta)
    torch.cuda.synchronize()
    _, scale, _ = reference(d, E, w.cpu().numpy(), beta, terms=oracle_terms(d))
    assert np.max(np.abs((a - b).cpu().numpy()) / scale) <= 1e-13


def test_complex_refusals():
    alpha = np.array([[1, 0], [1, 0], [1, 1]])
    eps = np.array([[1, 0], [1, 0], [0, 1]])
    T = amd.Terms(alpha, eps, 1, [1, 0], multipole=True)
    E = torch.zeros((8, 2), dtype=torch.complex128, device=DEV)
    w = torch.from_numpy(2j * np.pi * np.arange(1, 3) / 2.0).to(DEV)
    with pytest.raises(amd.AmiError) as e:
        amd.evaluate_complex(T, E, w, 2.0)
    assert e.value.code == -7
    with pytest.raises(amd.AmiError) as e:
        amd.evaluate_complex_adjoint(T, E, w, 2.0, grad_out=torch.ones((2, 8), dtype=torch.complex128, device=DEV))
    assert e.value.code == -7
    T2 = amd.Terms.from_diagram(order2_example())
    with pytest.raises(amd.AmiError) as e:
        amd.evaluate_complex(T2, torch.zeros((8, 3), dtype=torch.float64, device=DEV), w, 2.0)
    assert e.value.code == -1


@pytest.mark.parametrize("order,i,beta,n_e,e_reg", [
    (2, None, 5.0, 1000, 0.0), (3, 0, 2.0, 1500, 0.0), (4, 1, 5.0, 777, 0.0), (4, 6, 2.0, 600, 0.3),
    (5, 2, 5.0, 300, 0.0), (6, 0, 5.0, 90, 0.0),
])
@pytest.mark.parametrize("variant", [amd.VARIANT_AUTO, amd.VARIANT_SPECIALIZED, amd.VARIANT_TWO_PASS],
                         ids=["auto", "one_pass", "passes"])
def test_complex_adjoint_vs_oracle(order, i, beta, n_e, e_reg, variant):
    """dL/dRe E + i dL/dIm E per sample, dL/dbeta and dL/dw within 1e-10 of
    their rounding scales on samples away from poles; the values formed on the
    way equal amiEvaluateComplex's, and their row sums.  AUTO runs the one-pass
    kernel up to 512 terms and the passes above; the two forced variants run
    one each."""
    d = _diag(order, i)
    eta = 0.25 / (beta * d.n_int)
    E = complex_energies(n_e, d.n_eps, seed=(94, order, i or 0), a=3.0, eta=eta)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, -1.5, -1.5, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    n = len(E)
    rng = np.random.default_rng(95)
    cot = rng.standard_normal((len(w), n)) + 1j * rng.standard_normal((len(w), n))
    cot_sum = np.array([0.2 + 0.1j, -0.3j, 0.15])
    T = amd.Terms.from_diagram(d)
    T.set_variant(variant)
    Et, wt = torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV)
    out = torch.empty((len(w), n), dtype=torch.complex128, device=DEV)
    out_sum = torch.empty((len(w),), dtype=torch.complex128, device=DEV)
    g_e, g_b, g_w = amd.evaluate_complex_adjoint(T, Et, wt, beta, e_reg, grad_out=torch.from_numpy(cot).to(DEV),
                                                 grad_sum=torch.from_numpy(cot_sum).to(DEV), out=out,
                                                 out_sum=out_sum)
    passes = variant == amd.VARIANT_TWO_PASS or (variant == amd.VARIANT_AUTO and T.info()["T"] > 512)
    assert amd.last_variant() == ("specialized complex passes" if passes else "specialized complex")
    T.set_variant(amd.VARIANT_AUTO)
    fwd, _ = amd.evaluate_complex(T, Et, wt, beta, e_reg)
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized complex"
    full = cot + cot_sum[:, None]
    ref_e, ref_b, ref_w = gradients(terms, d.n_int, E, w, beta, full, e_reg)
    sc = gradient_scales(terms, d.n_int, E, w, beta, full, e_reg)
    ge = g_e.cpu().numpy()
    assert np.max(np.abs(ge - ref_e.astype(np.complex128)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(float(g_b) - float(ref_b)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(g_w.cpu().numpy() - ref_w.astype(np.complex128))) <= 1e-10 * sc["w"]
    got = out.cpu().numpy()
    ref, scale, dist = reference(d, E, w, beta, e_reg, terms=terms)
    check(got, ref, scale, dist, label=f"complex adjoint values order {order}")
    assert np.max(np.abs(got - fwd.cpu().numpy()) / scale) <= 1e-13
    np.testing.assert_allclose(out_sum.cpu().numpy(), got.sum(axis=1), rtol=1e-12, atol=1e-12 * scale.sum())


def test_complex_adjoint_real_limit_and_empty():
    """At real energies (given as complex numbers) the real part of the energy
    gradient, dL/dbeta and dL/dw equal amiEvaluateAdjoint's up to rounding;
    no samples give zero reductions."""
    d = random_self_energy(4, (0, 4, 3))
    T = amd.Terms.from_diagram(d)
    beta = 5.0
    E = uniform_energies(1100, d.n_eps, seed=96, a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    cot = np.random.default_rng(97).standard_normal((len(w), len(E))) + 0.5j
    Er, wt, ct = torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(cot).to(DEV)
    ra, rb, rw = amd.evaluate_adjoint(T, Er, wt, beta, grad_out=ct)
    ca, cb, cw = amd.evaluate_complex_adjoint(T, Er.to(torch.complex128), wt, beta, grad_out=ct)
    torch.cuda.synchronize()
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot)
    assert np.max(np.abs(ca.real.cpu().numpy() - ra.cpu().numpy()) / np.maximum(sc["E"], 1e-300)) <= 1e-12
    assert abs(float(cb) - float(rb)) <= 1e-12 * sc["beta"]
    assert np.max(np.abs((cw - rw).cpu().numpy())) <= 1e-12 * sc["w"]
    z = torch.zeros((0, d.n_eps), dtype=torch.complex128, device=DEV)
    g0, b0, w0 = amd.evaluate_complex_adjoint(T, z, wt, beta, grad_sum=torch.ones(len(w), dtype=torch.complex128,
                                                                                    device=DEV))
    torch.cuda.synchronize()
    assert g0.shape == (0, d.n_eps) and float(b0) == 0.0 and torch.all(w0 == 0)


@pytest.mark.parametrize("order,seed,n_e", [(4, (0, 4, 1), 3000), (6, (0, 6, 0), 700), (6, (5, 6, 2), 1100)])
def test_complex_two_pass(order, seed, n_e):
    """The two-pass complex forward against the oracle: forced at orders 4 and
    6 (where the one-pass kernel also serves: equal to it up to rounding), and
    by AUTO at order 6 with 2804 terms (above the one-pass size); the samples
    in one chunk and in several (a ragged last one), bitwise alike."""
    d = random_self_energy(order, seed)
    T = amd.Terms.from_diagram(d)
    big = T.info()["T"] > 1024
    if not big:
        T.set_variant(amd.VARIANT_TWO_PASS)
    beta, e_reg = 5.0, 0.02
    eta = 0.25 / (beta * d.n_int)
    E = complex_energies(n_e, d.n_eps, seed=(98, order), a=3.0, eta=eta)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -3.0, 3.0, 0.05)])
    Et, wt = torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV)
    out, s = amd.evaluate_complex(T, Et, wt, beta, e_reg, want_out=True, want_sum=True)
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized complex two-pass"
    cols = 2 * (T.info()["G"] + d.n_eps)
    try:
        amd.set_two_pass_chunk_bytes(max(1 << 16, 256 * 8 * cols * 2))     # chunks of 512 samples
        out2, s2 = amd.evaluate_complex(T, Et, wt, beta, e_reg, want_out=True, want_sum=True)
        torch.cuda.synchronize()
    finally:
        amd.set_two_pass_chunk_bytes(1 << 30)
    assert torch.equal(out, out2) and torch.equal(s, s2)
    got = out.cpu().numpy()
    ref, scale, dist = reference(d, E, w, beta, e_reg)
    check(got, ref, scale, dist, label=f"complex two-pass order {order}")
    np.testing.assert_allclose(s.cpu().numpy(), got.sum(axis=1), rtol=1e-12, atol=1e-12 * scale.sum())
    if not big:
        T.set_variant(amd.VARIANT_AUTO)
        one, _ = amd.evaluate_complex(T, Et, wt, beta, e_reg)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized complex"
        assert np.max(np.abs(one.cpu().numpy() - got) / scale) <= 1e-13


@pytest.mark.parametrize("order,seed,n_e", [(5, (0, 5, 0), 1100), (6, (5, 6, 2), 300)])
def test_complex_adjoint_passes_chunks_and_large(order, seed, n_e):
    """The adjoint at complex energies in passes: at order 6 with 2804 terms
    (beyond the one-pass kernel), the samples in one chunk and in several (a
    ragged last one) and two frequency rows, bitwise alike, against the
    oracle's gradients (on a sampled subset at 2804 terms)."""
    d = random_self_energy(order, seed)
    T = amd.Terms.from_diagram(d)
    T.set_variant(amd.VARIANT_TWO_PASS)      # AUTO takes the one-pass kernel at 264 terms
    beta, e_reg = 5.0, 0.02
    eta = 0.25 / (beta * d.n_int)
    E = complex_energies(n_e, d.n_eps, seed=(99, order), a=3.0, eta=eta)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(1, -1.5, -1.5, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    n = len(E)
    rng = np.random.default_rng(100)
    cot = rng.standard_normal((len(w), n)) + 1j * rng.standard_normal((len(w), n))
    Et, wt, ct = torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(cot).to(DEV)

    def run():
        out = torch.empty((len(w), n), dtype=torch.complex128, device=DEV)
        g = amd.evaluate_complex_adjoint(T, Et, wt, beta, e_reg, grad_out=ct, out=out)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized complex passes"
        return [x.cpu().numpy() for x in g] + [out.cpu().numpy()]

    one = run()
    cols = 4 * (T.info()["G"] + d.n_eps)
    try:
        amd.set_two_pass_chunk_bytes(max(1 << 16, 256 * 8 * cols * 2))     # chunks of 512 samples
        many = run()
    finally:
        amd.set_two_pass_chunk_bytes(1 << 30)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
    g_e, g_b, g_w, out = one
    pick = np.arange(n) if n <= 400 else np.random.default_rng(101).choice(n, 400, replace=False)
    sub = np.sort(pick[:40]) if order == 6 else np.sort(pick)
    ref_e, _, _ = gradients(terms, d.n_int, E[sub], w, beta, cot[:, sub], e_reg)
    sc = gradient_scales(terms, d.n_int, E[sub], w, beta, cot[:, sub], e_reg)
    assert np.max(np.abs(g_e[sub] - ref_e.astype(np.complex128)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    if order < 6:                       # the reductions over every sample
        _, ref_b, ref_w = gradients(terms, d.n_int, E, w, beta, cot, e_reg)
        scf = gradient_scales(terms, d.n_int, E, w, beta, cot, e_reg)
        assert abs(float(g_b) - float(ref_b)) <= 1e-10 * scf["beta"]
        assert np.max(np.abs(g_w - ref_w.astype(np.complex128))) <= 1e-10 * scf["w"]
    ref, scale, dist = reference(d, E[sub], w, beta, e_reg, terms=terms)
    check(out[:, sub], ref, scale, dist, label=f"complex adjoint passes values order {order}")


def test_complex_autograd_gradcheck():
    """AmiEvaluateComplex through torch's gradient check at complex energies
    (torch takes complex inputs' gradients as dL/dRe + i dL/dIm), beta as a
    host tensor, a Matsubara and a real frequency."""
    from paper_2311_17189_amd.autograd import AmiEvaluateComplex
    d = random_self_energy(3, (0, 3, 1))
    T = amd.Terms.from_diagram(d)
    E = torch.from_numpy(complex_energies(6, d.n_eps, seed=102, a=2.0, eta=0.05)).to(DEV).requires_grad_(True)
    w = torch.tensor([[1j * np.pi / 2.0], [0.3 + 0.1j]], dtype=torch.complex128, device=DEV, requires_grad=True)
    beta = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda e, ww, b: AmiEvaluateComplex.apply(T, e, ww, b), (E, w, beta),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("variant", [amd.VARIANT_AUTO, amd.VARIANT_TWO_PASS], ids=["one_pass", "passes"])
def test_complex_adjoint_strided_inputs(variant):
    """Energies read from a strided view and from a transposed one give the
    same bits as a contiguous copy, in one pass and in passes."""
    d = random_self_energy(3, (0, 3, 0))
    T = amd.Terms.from_diagram(d)
    T.set_variant(variant)
    beta = 3.0
    big = complex_energies(777, d.n_eps + 3, seed=103, a=3.0, eta=0.03)
    w = torch.from_numpy(np.concatenate([matsubara_freqs(1, beta), real_freqs(1, 0.5, 0.5, 0.05)])).to(DEV)
    Eb = torch.from_numpy(big).to(DEV)
    views = [Eb[:, 1:1 + d.n_eps], Eb[:, 1:1 + d.n_eps].contiguous(),
             Eb[:, 1:1 + d.n_eps].contiguous().t().contiguous().t()]
    assert views[0].stride() == (d.n_eps + 3, 1) and views[2].stride() == (1, 777)
    cot = torch.from_numpy(np.random.default_rng(104).standard_normal((2, 777)) + 0.3j).to(DEV)
    res = []
    for E in views:
        out = torch.empty((2, 777), dtype=torch.complex128, device=DEV)
        g = amd.evaluate_complex_adjoint(T, E, w, beta, grad_out=cot, out=out)
        torch.cuda.synchronize()
        res.append([x.cpu() for x in g] + [out.cpu()])
    assert amd.last_variant() == ("specialized complex passes" if variant == amd.VARIANT_TWO_PASS
                                  else "specialized complex")
    for r in res[1:]:
        for a, b in zip(res[0], r):
            assert torch.equal(a, b)
