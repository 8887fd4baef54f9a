"""GPU adjoint: the HIP adjoint kernels (through the C ABI) against the
oracle's analytic gradients and against central finite differences of the HIP
forward evaluation in float64 (step 1e-6)."""
import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, order2_example,
                        random_self_energy, real_freqs, uniform_energies)
from oracle.evaluate import (energies_from_k, gradients, momentum_gradients, term_magnitudes)

from parity import check, far_from_poles, gradient_scale, gradient_scales, oracle_terms, reference

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"

VARIANTS = pytest.mark.parametrize("variant", [amd.VARIANT_PACKED, amd.VARIANT_SPECIALIZED],
                                   ids=["packed", "specialized"])
# the adjoint's kernels: table-driven, specialized in one pass, specialized in
# passes over a workspace (VARIANT_TWO_PASS; AUTO above 128 terms)
ADJ_VARIANTS = pytest.mark.parametrize("variant", [amd.VARIANT_PACKED, amd.VARIANT_SPECIALIZED,
                                                   amd.VARIANT_TWO_PASS],
                                       ids=["packed", "specialized", "passes"])


def _terms(d, variant=amd.VARIANT_AUTO):
    t = amd.Terms.from_diagram(d)
    t.set_variant(variant)
    return t


def _cot(n_f, n_e, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_f, n_e)) + 1j * rng.standard_normal((n_f, n_e))


def _rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("order,i,beta", [(2, None, 5.0), (3, 1, 2.0), (4, 1, 5.0), (4, 1, 20.0),
                                          (5, 0, 3.0), (6, 0, 5.0)])
@ADJ_VARIANTS
def test_energy_adjoint_vs_oracle(order, i, beta, variant):
    """Per-sample dL/dE within 1e-10 of sum_t |dL_t/dE| (1e-6 next to a pole of
    one term); the sums over samples (dL/dbeta, dL/dw) within 1e-10 relative
    on samples away from poles."""
    d = order2_example() if i is None else random_self_energy(order, (0, order, i))
    n_e = 300 if order < 6 else 60
    E = uniform_energies(n_e, d.n_eps, seed=(20, order), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 1.0, 1.0, 0.05)])
    terms = oracle_terms(d)
    cot = _cot(len(w), n_e, 1)
    cot_sum = np.array([0.5 - 0.25j, 0.1j, -0.3])
    T = _terms(d, variant)
    g_e, _, _ = amd.evaluate_adjoint(T, torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), beta,
                                     grad_out=torch.from_numpy(cot).to(DEV),
                                     grad_sum=torch.from_numpy(cot_sum).to(DEV))
    torch.cuda.synchronize()
    full = cot + cot_sum[:, None]
    ref_e, _, _ = gradients(terms, d.n_int, E, w, beta, full)
    scale = gradient_scale(terms, d.n_int, E, w, beta, full)
    err = np.abs(g_e.cpu().numpy() - ref_e.astype(np.float64)) / np.maximum(scale, 1e-300)
    keep = far_from_poles(terms, d.n_int, E, w)
    near = np.setdiff1d(np.arange(n_e), keep)
    assert err[keep].max() <= 1e-10
    if len(near):
        assert err[near].max() <= 1e-6
    # reductions over samples, on samples away from poles
    Ek = np.ascontiguousarray(E[keep])
    ck = np.ascontiguousarray(cot[:, keep])
    _, g_b, g_w = amd.evaluate_adjoint(T, torch.from_numpy(Ek).to(DEV), torch.from_numpy(w).to(DEV), beta,
                                       grad_out=torch.from_numpy(ck).to(DEV),
                                       grad_sum=torch.from_numpy(cot_sum).to(DEV))
    torch.cuda.synchronize()
    _, ref_b, ref_w = gradients(terms, d.n_int, Ek, w, beta, ck + cot_sum[:, None])
    sc = gradient_scales(terms, d.n_int, Ek, w, beta, ck + cot_sum[:, None])
    assert abs(float(g_b) - float(ref_b)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(g_w.cpu().numpy() - ref_w.astype(np.complex128))) <= 1e-10 * sc["w"]


@pytest.mark.parametrize("order,i", [(2, None), (4, 1), (4, 3), (5, 2)])
@ADJ_VARIANTS
def test_hubbard_adjoint_vs_oracle(order, i, variant):
    """Momentum-path adjoint: every output within 1e-10 of its rounding scale
    (the sum over terms, and over samples for reduced outputs, of the
    single-term contributions' magnitudes), on samples away from poles."""
    d = order2_example() if i is None else random_self_energy(order, (0, order, i))
    beta, t, mu = 5.0, 1.0, 0.1
    n_e = 500
    k = k_samples(n_e, d.n_int, seed=(21, order))
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu), w)
    k = np.ascontiguousarray(k[keep])
    n_e = len(keep)
    cot = _cot(1, n_e, 2)
    T = _terms(d, variant)
    g_k, g_mu, g_t, g_b, g_w = amd.evaluate_hubbard_adjoint(
        T, torch.from_numpy(k).to(DEV), q, t, mu, torch.from_numpy(w).to(DEV), beta,
        grad_out=torch.from_numpy(cot).to(DEV))
    torch.cuda.synchronize()
    E = energies_from_k(d.alpha, k, q, t, mu)
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, hubbard=(d.alpha, k, q, t, mu))
    err_k = np.abs(g_k.cpu().numpy() - dk.astype(np.float64)) / np.maximum(sc["k"], 1e-300)
    assert err_k.max() <= 1e-10
    for got, ref, name in ((g_mu, dmu, "mu"), (g_t, dt, "t"), (g_b, db, "beta")):
        assert abs(float(got) - float(ref)) <= 1e-10 * sc[name], name
    assert np.max(np.abs(g_w.cpu().numpy() - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


@VARIANTS
def test_adjoint_matches_finite_differences_of_forward(variant):
    """Central differences (h = 1e-6, float64) of the HIP forward row sum with
    respect to mu, t, beta and a real frequency, against the HIP adjoint."""
    d = random_self_energy(4, (0, 4, 1))
    beta, t, mu = 5.0, 1.0, 0.05
    q = np.array(DEFAULT_Q)
    omega, gamma = 0.7, 0.05
    kh = k_samples(20000, d.n_int, seed=22)
    # keep samples whose single-term poles are far away: central differences
    # need the third derivative to stay moderate within +-h
    keep = far_from_poles(oracle_terms(d), d.n_int, energies_from_k(d.alpha, kh, q, t, mu),
                          np.array([omega + 1j * gamma]), near=1e-2)
    k = torch.from_numpy(np.ascontiguousarray(kh[keep])).to(DEV)
    n_e = len(keep)
    T = _terms(d, variant)

    def loss(tt, mm, bb, om):
        w = torch.tensor([om + 1j * gamma], dtype=torch.complex128, device=DEV)
        _, s = amd.evaluate_hubbard(T, k, q, tt, mm, w, bb, want_out=False, want_sum=True)
        return float(s.real.sum().item())

    w = torch.tensor([omega + 1j * gamma], dtype=torch.complex128, device=DEV)
    gs = torch.ones(1, dtype=torch.complex128, device=DEV)
    _, g_mu, g_t, g_b, g_w = amd.evaluate_hubbard_adjoint(T, k, q, t, mu, w, beta, grad_sum=gs)
    h = 1e-6
    checks = [
        (float(g_mu), (loss(t, mu + h, beta, omega) - loss(t, mu - h, beta, omega)) / (2 * h)),
        (float(g_t), (loss(t + h, mu, beta, omega) - loss(t - h, mu, beta, omega)) / (2 * h)),
        (float(g_b), (loss(t, mu, beta + h, omega) - loss(t, mu, beta - h, omega)) / (2 * h)),
        (float(g_w[0, 0].real), (loss(t, mu, beta, omega + h) - loss(t, mu, beta, omega - h)) / (2 * h)),
    ]
    # the difference quotient's own rounding: each loss carries an error of a
    # few ulp of sum_s sum_t |v_t| (the scale of the sum it rounds), divided by 2h
    E = energies_from_k(d.alpha, kh[keep], q, t, mu)
    mag = float(np.sum(term_magnitudes(oracle_terms(d), d.n_int, E, np.array([omega + 1j * gamma]), beta)))
    floor = 8 * 2.0 ** -52 * mag / (2 * h)
    for got, fd in checks:
        assert abs(got - fd) <= 1e-7 * abs(fd) + floor, (got, fd, floor)


@ADJ_VARIANTS
def test_momentum_gradient_matches_finite_differences(variant):
    """Every momentum component of the order-4 adjoint step (8 per sample)
    against central differences (h = 1e-6, float64) of the HIP forward: each
    component is moved in every sample at once (samples are independent), so
    16 forward calls give the difference quotient of every (sample, component).
    The bar is 1e-7 relative plus the quotient's own rounding (a few ulp of
    sum_t |v_t| over 2h); samples within 0.05 of a pole of one term are left
    out (the third derivative there outgrows the step)."""
    d = random_self_energy(4, (0, 4, 1))
    beta, t, mu = 5.0, 1.0, 0.0
    q = np.array(DEFAULT_Q)
    wv = matsubara_freqs(1, beta)
    kh = k_samples(6000, d.n_int, seed=(27, 4))
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, energies_from_k(d.alpha, kh, q, t, mu), wv, near=0.05)
    kk = np.ascontiguousarray(kh[keep])
    n_e = len(kk)
    assert n_e > 2000
    cot = _cot(1, n_e, 28)
    T = _terms(d, variant)
    w = torch.from_numpy(wv).to(DEV)
    kt = torch.from_numpy(kk).to(DEV)
    g_k, *_ = amd.evaluate_hubbard_adjoint(T, kt, q, t, mu, w, beta, grad_out=torch.from_numpy(cot).to(DEV))
    g_k = g_k.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(kk)
    for c in range(2 * d.n_int):
        plus, minus = kk.copy(), kk.copy()
        plus[:, c] += h
        minus[:, c] -= h
        op, _ = amd.evaluate_hubbard(T, torch.from_numpy(plus).to(DEV), q, t, mu, w, beta)
        om, _ = amd.evaluate_hubbard(T, torch.from_numpy(minus).to(DEV), q, t, mu, w, beta)
        dq = (op.cpu().numpy() - om.cpu().numpy()) / (2 * h)
        fd[:, c] = np.real(np.conj(cot) * dq).sum(axis=0)
    E = energies_from_k(d.alpha, kk, q, t, mu)
    mag = (np.abs(cot) * term_magnitudes(terms, d.n_int, E, wv, beta).astype(np.float64)).sum(axis=0)
    floor = 8 * 2.0 ** -52 * mag / (2 * h)
    err = np.abs(g_k - fd)
    bound = 1e-7 * np.abs(fd) + floor[:, None]
    assert np.all(err <= bound), float(np.max(err / bound))
    # where the quotient's rounding is below a tenth of the bar, the plain
    # relative error is within 1e-7 itself
    clean = floor[:, None] <= 1e-8 * np.abs(fd)
    worst = float(np.max(err[clean] / np.abs(fd[clean]))) if clean.any() else 0.0
    print(f"k-gradient vs FD: {int(clean.sum())} of {fd.size} entries under the plain bar, worst {worst:.2e}")
    assert clean.sum() > n_e // 2
    assert worst <= 1e-7


def test_autograd_function_gradcheck():
    from paper_2311_17189_amd.autograd import AmiHubbard
    d = order2_example()
    T = amd.Terms.from_diagram(d)
    k = torch.from_numpy(k_samples(5, 2, seed=23)).to(DEV).requires_grad_(True)
    q = np.array(DEFAULT_Q)
    # the scalars as host tensors (read without a device synchronization)
    t = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
    beta = torch.tensor(3.0, dtype=torch.float64, requires_grad=True)
    w = torch.tensor([[0.4 + 0.3j], [1j * np.pi / 3.0]], dtype=torch.complex128, device=DEV,
                     requires_grad=True)

    def f(k_, t_, mu_, w_, b_):
        out, s = AmiHubbard.apply(T, k_, q, t_, mu_, w_, b_)
        return out, s

    assert torch.autograd.gradcheck(f, (k, t, mu, w, beta), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_autograd_with_number_scalars_and_device_scalars():
    """t and mu as plain numbers get no gradient and break nothing; beta as a
    CUDA tensor gets its gradient on the device; k's gradient equals the
    adjoint call's."""
    from paper_2311_17189_amd.autograd import AmiHubbard
    d = random_self_energy(3, (0, 3, 1))
    T = amd.Terms.from_diagram(d)
    q = np.array(DEFAULT_Q)
    k = torch.from_numpy(k_samples(300, d.n_int, seed=26)).to(DEV).requires_grad_(True)
    w = torch.from_numpy(matsubara_freqs(2, 4.0)).to(DEV)
    beta = torch.tensor(4.0, dtype=torch.float64, device=DEV, requires_grad=True)
    out, s = AmiHubbard.apply(T, k, q, 1.0, 0.1, w, beta)
    s.real.sum().backward()
    gs = torch.ones(2, dtype=torch.complex128, device=DEV)
    g_k, _, _, g_b, _ = amd.evaluate_hubbard_adjoint(T, k.detach(), q, 1.0, 0.1, w, 4.0, grad_sum=gs)
    torch.cuda.synchronize()
    assert torch.equal(k.grad, g_k)
    assert beta.grad.device == beta.device and torch.equal(beta.grad, g_b)


def test_autograd_energy_function():
    from paper_2311_17189_amd.autograd import AmiEvaluate
    d = random_self_energy(3, (0, 3, 1))
    T = amd.Terms.from_diagram(d)
    E = torch.from_numpy(uniform_energies(6, d.n_eps, seed=24, a=2.0)).to(DEV).requires_grad_(True)
    w = torch.tensor([[1j * np.pi / 2.0]], dtype=torch.complex128, device=DEV, requires_grad=True)
    beta = torch.tensor(2.0, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda e, ww, b: AmiEvaluate.apply(T, e, ww, b), (E, w, beta),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


def test_adjoint_deterministic_and_sum_cotangent():
    d = random_self_energy(4, (0, 4, 2))
    beta = 5.0
    n_e = 3000
    E = torch.from_numpy(uniform_energies(n_e, d.n_eps, seed=25, a=4.0)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(2, beta)).to(DEV)
    T = amd.Terms.from_diagram(d)
    gs = torch.tensor([1.0 + 0.5j, -0.25j], dtype=torch.complex128, device=DEV)
    a = amd.evaluate_adjoint(T, E, w, beta, grad_sum=gs)
    b = amd.evaluate_adjoint(T, E, w, beta, grad_sum=gs)
    # the row-sum cotangent equals a broadcast per-sample cotangent
    c = amd.evaluate_adjoint(T, E, w, beta, grad_out=gs[:, None].expand(2, n_e).contiguous())
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for x, y in zip(a, c):
        assert torch.allclose(x, y, rtol=1e-13, atol=0)


def test_kernel_variants_agree():
    """Every forward variant -- double tables, packed, specialized (one or two
    passes), and the automatic choice -- meets the parity bar against the
    oracle on the same inputs, and the automatic choice names what it ran."""
    for order, i in ((3, 0), (4, 1), (5, 2), (6, 1)):
        d = random_self_energy(order, (0, order, i))
        beta = 5.0
        n_e = 777 if order < 6 else 200
        Eh = uniform_energies(n_e, d.n_eps, seed=(26, order), a=4.0)
        wh = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -3, 3, 0.05)])
        E = torch.from_numpy(Eh).to(DEV)
        w = torch.from_numpy(wh).to(DEV)
        T = amd.Terms.from_diagram(d)
        ref, scale, dist = reference(d, Eh, wh, beta)
        names = {}
        inf = T.info()
        small = inf["T"] <= 1024
        # the specialized forward runs in two passes where the one-pass kernel
        # would not hold its groups and reciprocals in registers
        two = inf["T"] > 1024 or 2 * inf["G"] + 4 * inf["D"] > 128
        variants = [amd.VARIANT_TABLES, amd.VARIANT_PACKED, amd.VARIANT_AUTO, amd.VARIANT_TWO_PASS]
        if small:
            variants.append(amd.VARIANT_SPECIALIZED)
        for v in variants:
            T.set_variant(v)
            o, _ = amd.evaluate(T, E, w, beta)
            names[v] = amd.last_variant()
            torch.cuda.synchronize()
            check(o.cpu().numpy(), ref, scale, dist, label=f"variant {v} order {order}")
        assert names[amd.VARIANT_TABLES] == "double tables"
        assert names[amd.VARIANT_PACKED].startswith("packed self-energy")
        assert names[amd.VARIANT_TWO_PASS] == "specialized two-pass"
        want = "specialized two-pass" if two else "specialized"
        assert names[amd.VARIANT_AUTO] == want
        if small:
            assert names[amd.VARIANT_SPECIALIZED] == want


def test_adjoint_empty_batch():
    d = order2_example()
    T = amd.Terms.from_diagram(d)
    E = torch.zeros((0, 3), dtype=torch.float64, device=DEV)
    w = torch.from_numpy(matsubara_freqs(1, 2.0)).to(DEV)
    g_e, g_b, g_w = amd.evaluate_adjoint(T, E, w, 2.0, grad_sum=torch.ones(1, dtype=torch.complex128,
                                                                            device=DEV))
    torch.cuda.synchronize()
    assert g_e.shape == (0, 3) and float(g_b) == 0.0 and torch.all(g_w == 0)


@VARIANTS
def test_value_and_gradient_in_one_pass(variant):
    """The adjoint entry points also return the forward values when asked: the
    energy path bitwise equal to amiEvaluate, the momentum path within the
    parity bar (its energies come from the sin/cos pair instead of cos alone)."""
    d = random_self_energy(4, (0, 4, 2))
    beta = 5.0
    T = _terms(d, variant)
    E = torch.from_numpy(uniform_energies(1500, d.n_eps, seed=27, a=4.0)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(2, beta)).to(DEV)
    gs = torch.tensor([1.0, 0.5j], dtype=torch.complex128, device=DEV)
    out = torch.empty((2, 1500), dtype=torch.complex128, device=DEV)
    out_sum = torch.empty((2,), dtype=torch.complex128, device=DEV)
    g1 = amd.evaluate_adjoint(T, E, w, beta, grad_sum=gs, out=out, out_sum=out_sum)
    g2 = amd.evaluate_adjoint(T, E, w, beta, grad_sum=gs)
    ref, ref_sum = amd.evaluate(T, E, w, beta, want_sum=True)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert torch.allclose(out_sum, ref_sum, rtol=1e-12)
    for x, y in zip(g1, g2):
        assert torch.equal(x, y)
    # momentum path
    k = k_samples(1200, d.n_int, seed=28)
    q = np.array(DEFAULT_Q)
    wh = np.concatenate([matsubara_freqs(1, beta), real_freqs(1, 0.3, 0.3, 0.05)])
    out = torch.empty((2, 1200), dtype=torch.complex128, device=DEV)
    amd.evaluate_hubbard_adjoint(T, torch.from_numpy(k).to(DEV), q, 1.0, 0.0, torch.from_numpy(wh).to(DEV),
                                 beta, grad_sum=gs, out=out)
    torch.cuda.synchronize()
    from parity import reference_hubbard
    ref, scale, dist, _ = reference_hubbard(d, k, q, 1.0, 0.0, wh, beta)
    check(out.cpu().numpy(), ref, scale, dist, label="value and gradient")


def test_auto_adjoint_above_its_one_pass_limit():
    """AUTO runs the specialized adjoint in one pass up to 128 terms and in
    passes over a workspace above (the forward of a solution above 1024 terms
    in two passes); a forced variant that cannot serve the call fails it."""
    small = amd.Terms.from_diagram(random_self_energy(4, (0, 4, 1)))
    large = amd.Terms.from_diagram(random_self_energy(5, (0, 5, 0)))
    huge = amd.Terms.from_diagram(random_self_energy(6, (5, 6, 0)))
    beta = 5.0
    w = torch.from_numpy(matsubara_freqs(1, beta)).to(DEV)
    gs = torch.ones(1, dtype=torch.complex128, device=DEV)
    for T, want in ((small, "specialized"), (large, "specialized passes")):
        E = torch.from_numpy(uniform_energies(100, T.info()["n_eps"], seed=29, a=3.0)).to(DEV)
        amd.evaluate_adjoint(T, E, w, beta, grad_sum=gs)
        assert amd.last_variant() == want, amd.last_variant()
    E = torch.from_numpy(uniform_energies(50, huge.info()["n_eps"], seed=30, a=3.0)).to(DEV)
    amd.evaluate(huge, E, w, beta)
    assert amd.last_variant() == "specialized two-pass"
    amd.evaluate_adjoint(huge, E, w, beta, grad_sum=gs)
    assert amd.last_variant() == "specialized passes"
    huge.set_variant(amd.VARIANT_SPECIALIZED)
    with pytest.raises(amd.AmiError):
        amd.evaluate_adjoint(huge, E, w, beta, grad_sum=gs)
    huge.set_variant(amd.VARIANT_TABLES)
    with pytest.raises(amd.AmiError):
        amd.evaluate_adjoint(huge, E, w, beta, grad_sum=gs)


@pytest.mark.parametrize("order,seed", [(5, (0, 5, 0)), (6, (5, 6, 2))])
def test_adjoint_passes_chunks_rows_and_values(order, seed):
    """The adjoint in passes with the samples in several workspace chunks (a
    ragged last one) and three frequency rows (the group-sum cotangents added
    to the stored ones after the first row): gradients and the values it
    returns on the way against the oracle, the same bits as one chunk, and
    the same bits on a repeat."""
    d = random_self_energy(order, seed)
    beta = 5.0
    n_e = 1100 if order == 5 else 300
    Eh = uniform_energies(n_e, d.n_eps, seed=(31, order), a=3.0)
    wh = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.9, 0.9, 0.05)])
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, Eh, wh)
    Eh = np.ascontiguousarray(Eh[keep])
    n_e = len(Eh)
    cot = _cot(len(wh), n_e, 32)
    cot_sum = np.array([0.2 - 0.1j, 0.3j, -0.4])
    T = amd.Terms.from_diagram(d)
    E = torch.from_numpy(Eh).to(DEV)
    w = torch.from_numpy(wh).to(DEV)

    def run():
        out = torch.empty((len(wh), n_e), dtype=torch.complex128, device=DEV)
        out_sum = torch.empty((len(wh),), dtype=torch.complex128, device=DEV)
        g = amd.evaluate_adjoint(T, E, w, beta, grad_out=torch.from_numpy(cot).to(DEV),
                                 grad_sum=torch.from_numpy(cot_sum).to(DEV), out=out, out_sum=out_sum)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized passes"
        return [x.cpu().numpy() for x in g] + [out.cpu().numpy(), out_sum.cpu().numpy()]

    one = run()
    cols = 2 * T.info()["G"] + 2 * d.n_eps
    try:
        amd.set_two_pass_chunk_bytes(max(1 << 16, 256 * 8 * cols * 2))   # chunks of 512 samples
        many = run()
        again = run()
    finally:
        amd.set_two_pass_chunk_bytes(1 << 30)
    for a, b, c in zip(one, many, again):
        assert np.array_equal(a, b) and np.array_equal(b, c)
    g_e, g_b, g_w, out, out_sum = many
    full = cot + cot_sum[:, None]
    ref_e, ref_b, ref_w = gradients(terms, d.n_int, Eh, wh, beta, full)
    sc = gradient_scales(terms, d.n_int, Eh, wh, beta, full)
    assert np.max(np.abs(g_e - ref_e.astype(np.float64)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(float(g_b) - float(ref_b)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(g_w - ref_w.astype(np.complex128))) <= 1e-10 * sc["w"]
    ref, scale, dist = reference(d, Eh, wh, beta, terms=terms)
    check(out, ref, scale, dist, label=f"passes values order {order}")
    assert np.allclose(out_sum, out.sum(axis=1), rtol=1e-12, atol=1e-14 * float(scale.sum()))
