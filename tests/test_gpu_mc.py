"""Monte-Carlo integration on the GPU (amiIntegrateHubbard): momenta drawn in
the kernel from the counter-based generator, summed over samples, against the
oracle on the same draws; determinism; frequency chunks; the integrand class
and its estimate against a quadrature of the same integral."""
import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, matsubara_freqs, order2_example, random_self_energy, real_freqs
from oracle.evaluate import energies_from_k, evaluate_terms
from oracle.mc import draw_momenta

from parity import NEAR, TOL, TOL_NEAR, oracle_terms, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


@pytest.mark.parametrize("order,i,n,seed", [(2, None, 30011, 5), (4, 1, 20000, (1 << 40) + 7),
                                            (4, 3, 3333, 12)])
def test_mc_sums_match_oracle_on_the_same_draws(order, i, n, seed):
    d = order2_example() if i is None else random_self_energy(order, (0, order, i))
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    T = amd.Terms.from_diagram(d)
    sums = amd.integrate_hubbard(T, n, seed, q, t, mu, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    got = sums.cpu().numpy()
    k = draw_momenta(0, n, 2 * d.n_int, seed)
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta)
    tol = np.where(dist >= NEAR, TOL, TOL_NEAR) * scale                 # per (frequency, sample)
    want = np.stack([ref.real.sum(1), ref.imag.sum(1), (ref.real ** 2).sum(1), (ref.imag ** 2).sum(1)], axis=1)
    bound = np.stack([tol.sum(1), tol.sum(1), (2 * np.abs(ref) * tol).sum(1), (2 * np.abs(ref) * tol).sum(1)],
                     axis=1)
    assert np.all(np.abs(got - want) <= bound + 1e-300), (got, want, bound)


@pytest.mark.parametrize("i,n,chunk", [(0, 600, 1 << 16), (9, 1500, 1 << 30)])
def test_mc_two_pass_for_large_solutions(i, n, chunk):
    """A solution evaluated in two passes (order 6): the first pass draws the
    momenta, the sums match the oracle on the same draws; several chunks."""
    d = random_self_energy(6, (5, 6, i))
    T = amd.Terms.from_diagram(d)
    inf = T.info()
    assert inf["T"] > 1024 or 2 * inf["G"] + 4 * inf["D"] > 128
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    amd.set_two_pass_chunk_bytes(chunk)
    try:
        sums = amd.integrate_hubbard(T, n, 9, q, t, mu, torch.from_numpy(w).to(DEV), beta)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized two-pass"
        again = amd.integrate_hubbard(T, n, 9, q, t, mu, torch.from_numpy(w).to(DEV), beta)
        torch.cuda.synchronize()
    finally:
        amd.set_two_pass_chunk_bytes(1 << 30)
    assert torch.equal(sums, again)
    got = sums.cpu().numpy()
    k = draw_momenta(0, n, 2 * d.n_int, 9)
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta)
    tol = np.where(dist >= NEAR, TOL, TOL_NEAR) * scale
    want = np.stack([ref.real.sum(1), ref.imag.sum(1), (ref.real ** 2).sum(1), (ref.imag ** 2).sum(1)], axis=1)
    bound = np.stack([tol.sum(1), tol.sum(1), (2 * np.abs(ref) * tol).sum(1), (2 * np.abs(ref) * tol).sum(1)],
                     axis=1)
    assert np.all(np.abs(got - want) <= bound + 1e-300), (got, want, bound)


def test_mc_deterministic_chunked_and_edge_sizes():
    d = random_self_energy(3, (0, 3, 0))
    T = amd.Terms.from_diagram(d)
    beta = 4.0
    q = np.array(DEFAULT_Q)
    w = torch.from_numpy(matsubara_freqs(10, beta)).to(DEV)
    a = amd.integrate_hubbard(T, 100000, 3, q, 1.0, 0.0, w, beta)
    b = amd.integrate_hubbard(T, 100000, 3, q, 1.0, 0.0, w, beta)
    c = amd.integrate_hubbard(T, 100000, 3, q, 1.0, 0.0, w[8:], beta)   # rows 8, 9 alone
    e = amd.integrate_hubbard(T, 100000, 4, q, 1.0, 0.0, w, beta)       # another seed
    z = amd.integrate_hubbard(T, 0, 3, q, 1.0, 0.0, w[:2], beta)
    one = amd.integrate_hubbard(T, 1, 3, q, 1.0, 0.0, w[:1], beta)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a[8:], c)
    assert not torch.equal(a, e)
    assert torch.all(z == 0)
    k = draw_momenta(0, 1, 2 * d.n_int, 3)
    ref, _, _, _ = reference_hubbard(d, k, q, 1.0, 0.0, matsubara_freqs(1, beta), beta)
    r = complex(ref[0, 0])
    np.testing.assert_allclose(one.cpu().numpy()[0], [r.real, r.imag, r.real ** 2, r.imag ** 2], rtol=1e-10)


def test_integrand_call_and_estimate_against_quadrature():
    """Order 2 (four momentum components): the GPU estimate over 2^22 draws
    against the periodic trapezoid rule on a 16^4 grid (converged to ~1e-7
    here), within four standard errors; the callable equals amiEvaluateHubbard."""
    from paper_2311_17189_amd.integrand import Integrand
    d = order2_example()
    terms = oracle_terms(d)
    beta, t, mu = 2.0, 1.0, 0.3
    q = np.array(DEFAULT_Q)
    w = np.array([1j * np.pi / beta, 3j * np.pi / beta])
    T = amd.Terms.from_diagram(d)
    f = Integrand(T, q, t, mu, torch.from_numpy(w).to(DEV), beta)
    kt = torch.from_numpy(draw_momenta(0, 777, 4, 1)).to(DEV)
    out = f(kt)
    ref, _ = amd.evaluate_hubbard(T, kt, q, t, mu, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    mean, err = f.integrate(1 << 22, seed=21)
    g = -np.pi + 2 * np.pi * np.arange(16) / 16
    grid = np.stack(np.meshgrid(g, g, g, g, indexing="ij"), axis=-1).reshape(-1, 4)
    E = energies_from_k(d.alpha, grid, q, t, mu, dtype=np.float64)
    quad = evaluate_terms(terms, d.n_int, E, w, beta, dtype=np.float64).astype(np.complex128).mean(axis=1)
    assert np.all(np.abs(mean.real - quad.real) < 4 * err[:, 0])
    assert np.all(np.abs(mean.imag - quad.imag) < 4 * err[:, 1])
    assert np.all(err[:, 0] < 1e-3 * np.abs(quad) + 1e-4)


def test_mc_argument_checks():
    d = order2_example()
    T = amd.Terms.from_diagram(d)
    w = torch.from_numpy(matsubara_freqs(9, 1.0)).to(DEV)
    lib = amd.load_library()
    s = torch.empty((9, 4), dtype=torch.float64, device=DEV)
    q = np.array(DEFAULT_Q)
    # nine rows in one call exceed the limit (the Python wrapper splits them)
    code = lib.amiIntegrateHubbard(T.handle, 10, 0, q.ctypes.data, 1.0, 0.0, w.data_ptr(), 9, 1.0, 0.0,
                                   s.data_ptr(), None)
    assert code == -1
    code = lib.amiIntegrateHubbard(T.handle, 10, 0, q.ctypes.data, 1.0, 0.0, w.data_ptr(), 1, -1.0, 0.0,
                                   s.data_ptr(), None)
    assert code == -1
