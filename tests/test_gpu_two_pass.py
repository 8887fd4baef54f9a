"""The two-pass specialized forward on the GPU against the oracle: large
solutions that AUTO sends there (order 6, up to 2804 terms), the forced
variant on small ones, several sample chunks, both inputs, poles of higher
order, row sums, and the frequency-row limit."""
import types

import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy, real_freqs,
                        uniform_energies)

from parity import check, oracle_terms, reference, reference_hubbard
from test_multipole_cpu import CASES as MULTIPOLE, _oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


@pytest.fixture
def small_chunks():
    amd.set_two_pass_chunk_bytes(1 << 16)        # a few hundred samples per chunk
    yield
    amd.set_two_pass_chunk_bytes(1 << 30)


@pytest.mark.parametrize("i,n_e", [(0, 1500), (2, 700), (4, 600)])
def test_auto_two_pass_on_large_solutions(i, n_e):
    d = random_self_energy(6, (5, 6, i))
    T = amd.Terms.from_diagram(d)
    assert T.info()["T"] > 1024
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    k = k_samples(n_e, d.n_int, seed=(98, i))
    out, s = amd.evaluate_hubbard(T, torch.from_numpy(k).to(DEV), q, t, mu, torch.from_numpy(w).to(DEV), beta,
                                  want_sum=True)
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized two-pass"
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta)
    got = out.cpu().numpy()
    check(got, ref, scale, dist, label=f"two-pass order 6 seed {i}")
    np.testing.assert_allclose(s.cpu().numpy(), got.sum(axis=1), rtol=1e-12, atol=1e-12 * scale.sum())


@pytest.mark.parametrize("order,i", [(3, 0), (4, 1), (5, 2)])
def test_forced_two_pass_chunks_match_one_pass_and_oracle(order, i, small_chunks):
    d = random_self_energy(order, (0, order, i))
    beta = 5.0
    q = np.array(DEFAULT_Q)
    w = torch.from_numpy(np.concatenate([matsubara_freqs(3, beta), real_freqs(2, -3.0, 3.0, 0.05)])).to(DEV)
    k_host = k_samples(3001, d.n_int, seed=(99, order, i))
    k = torch.from_numpy(k_host).to(DEV)
    T = amd.Terms.from_diagram(d)
    T.set_variant(amd.VARIANT_TWO_PASS)
    a, sa = amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True)
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized two-pass"
    T.set_variant(amd.VARIANT_SPECIALIZED)
    b, sb = amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True)
    torch.cuda.synchronize()
    ref, scale, dist, _ = reference_hubbard(d, k_host, q, 1.0, 0.0, w.cpu().numpy(), beta)
    check(a.cpu().numpy(), ref, scale, dist, label=f"forced two-pass order {order}")
    assert np.max(np.abs((a - b).cpu().numpy()) / scale) <= 1e-12
    np.testing.assert_allclose(sa.cpu().numpy(), sb.cpu().numpy(), rtol=1e-12, atol=1e-12 * scale.sum())
    # deterministic
    a2, sa2 = amd.evaluate_hubbard(_two(d), k, q, 1.0, 0.0, w, beta, want_sum=True)
    torch.cuda.synchronize()
    assert torch.equal(a, a2) and torch.equal(sa, sa2)


def _two(d):
    T = amd.Terms.from_diagram(d)
    T.set_variant(amd.VARIANT_TWO_PASS)
    return T


def test_two_pass_energy_input_strided_and_multipole(small_chunks):
    d = random_self_energy(6, (5, 6, 11))
    beta = 4.0
    big = uniform_energies(777, d.n_eps + 3, seed=100, a=3.0)
    Et = torch.from_numpy(big).to(DEV)[:, 2:2 + d.n_eps]
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.5, 0.5, 0.05)])
    T = _two(d)
    out, _ = amd.evaluate(T, Et, torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    E = np.ascontiguousarray(big[:, 2:2 + d.n_eps])
    ref, scale, dist = reference(d, E, w, beta, terms=oracle_terms(d))
    check(out.cpu().numpy(), ref, scale, dist, label="two-pass strided energies")
    # poles of higher order through the two passes
    alpha, eps, n_int, ferm = MULTIPOLE["o4"]
    Tm = amd.Terms(alpha, eps, n_int, ferm, multipole=True)
    Tm.set_variant(amd.VARIANT_TWO_PASS)
    Em = uniform_energies(900, eps.shape[1], seed=101, a=3.0)
    out, _ = amd.evaluate(Tm, torch.from_numpy(Em).to(DEV), torch.from_numpy(w).to(DEV), beta)
    torch.cuda.synchronize()
    ref, scale, dist = reference(types.SimpleNamespace(n_int=n_int), Em, w, beta, terms=_oracle(MULTIPOLE["o4"]))
    check(out.cpu().numpy(), ref, scale, dist, label="two-pass multipole")


def test_two_pass_refusals_and_frequency_limit():
    d = random_self_energy(4, (0, 4, 1))
    T = _two(d)
    E = torch.zeros((4, d.n_eps), dtype=torch.float64, device=DEV) + 0.3
    w = torch.from_numpy(matsubara_freqs(65536, 5.0)).to(DEV)
    with pytest.raises(amd.AmiError) as e:           # the second kernel's grid height
        amd.evaluate(T, E, w, 5.0)
    assert e.value.code == -7
    # the adjoint under this variant runs in passes, its frequency rows in a
    # loop of the kernel (no grid-height limit): many rows are taken
    E2 = torch.from_numpy(uniform_energies(64, d.n_eps, seed=(35, 4), a=3.0)).to(DEV)
    g_e, _, g_w = amd.evaluate_adjoint(T, E2, w, 5.0, grad_sum=torch.ones(len(w), dtype=torch.complex128, device=DEV))
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized passes"
    assert g_e.shape == (64, d.n_eps) and g_w.shape == (65536, 1) and torch.isfinite(g_w).all()
