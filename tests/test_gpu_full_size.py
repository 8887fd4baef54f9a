"""The workloads at their full size on the GPU, checked where the oracle can
follow one sample at a time and through properties that hold at any size:
the real-frequency continuation on a 256-point grid (10^6 k-samples, out of
4.1 GB) and the adjoint step (10^6 k-samples, values and every gradient in one
pass)."""
import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy, real_freqs
from oracle.evaluate import energies_from_k, gradients, momentum_gradients

from parity import check, far_from_poles, gradient_scales, oracle_terms, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"
N_E = 1_000_000


def _sampled(n_e, n, seed):
    idx = np.sort(np.random.default_rng(seed).choice(n_e, n, replace=False))
    idx[-1] = n_e - 1
    return idx


def test_full_size_real_frequency_grid():
    """Order-4 diagram, 10^6 k-samples, omega + i Gamma for 256 omega in
    [-6, 6] with Gamma = 0.05 (the frequency enters the denominators only):
    all 256 rows of 200 sampled samples against the oracle one by one, and the
    row sums against the sums of the returned rows."""
    d = random_self_energy(4, (0, 4, 1))
    beta, t, mu = 5.0, 1.0, 0.0
    k = k_samples(N_E, d.n_int, seed=(4, 4, 2))
    q = np.array(DEFAULT_Q)
    w = real_freqs(256, -6.0, 6.0, 0.05)
    T = amd.Terms.from_diagram(d)
    out, s = amd.evaluate_hubbard(T, torch.from_numpy(k).to(DEV), q, t, mu, torch.from_numpy(w).to(DEV), beta,
                                  want_sum=True)
    torch.cuda.synchronize()
    assert out.shape == (256, N_E)
    idx = _sampled(N_E, 200, 5)
    sub = out[:, torch.from_numpy(idx).to(DEV)].cpu().numpy()
    ref, scale, dist, _ = reference_hubbard(d, k[idx], q, t, mu, w, beta, terms=oracle_terms(d))
    st = {}
    check(sub, ref, scale, dist, label="full-size real-frequency grid", stats=st)
    print(f"real-frequency grid: {st}", flush=True)
    rows = out.sum(dim=1)
    torch.cuda.synchronize()
    np.testing.assert_allclose(s.cpu().numpy(), rows.cpu().numpy(), rtol=1e-9,
                               atol=1e-12 * float(torch.abs(out).sum()))
    assert bool(torch.isfinite(torch.view_as_real(out)).all())


def test_full_size_adjoint_step():
    """The benchmark's step at its size: order-4 diagram, 10^6 k-samples, one
    Matsubara frequency, L = Re(conj(c) sum_s out).  Sampled rows of dL/dk and
    of the values against the oracle; the gradients that are sums over samples
    (mu, t, beta, w) and the row sum against the sums of two calls on the
    halves of the samples."""
    d = random_self_energy(4, (0, 4, 1))
    beta, t, mu = 5.0, 1.0, 0.0
    k = k_samples(N_E, d.n_int, seed=(4, 4, 1))
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    c = 0.7 - 0.4j
    T = amd.Terms.from_diagram(d)
    kt = torch.from_numpy(k).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    gs = torch.tensor([c], dtype=torch.complex128, device=DEV)

    def step(kk):
        out = torch.empty((1, kk.shape[0]), dtype=torch.complex128, device=DEV)
        out_sum = torch.empty((1,), dtype=torch.complex128, device=DEV)
        g = amd.evaluate_hubbard_adjoint(T, kk, q, t, mu, wt, beta, grad_sum=gs, out=out, out_sum=out_sum)
        return out, out_sum, g

    out, out_sum, (g_k, g_mu, g_t, g_b, g_w) = step(kt)
    half = N_E // 2 + 77                   # neither half a whole number of tiles
    _, sa, (_, ma, ta, ba, wa) = step(kt[:half])
    _, sb, (_, mb, tb, bb, wb) = step(kt[half:])
    torch.cuda.synchronize()
    assert amd.last_variant() == "specialized"

    # sums over samples: the whole equals the two halves
    for whole, a, b, name in ((g_mu, ma, mb, "mu"), (g_t, ta, tb, "t"), (g_b, ba, bb, "beta"),
                              (g_w, wa, wb, "w"), (out_sum, sa, sb, "row sum")):
        x, y, z = (np.asarray(v.cpu().numpy(), dtype=np.complex128) for v in (whole, a, b))
        bound = 1e-10 * max(np.max(np.abs(y)), np.max(np.abs(z)))
        assert np.max(np.abs(x - (y + z))) <= bound, name

    # sampled rows against the oracle
    idx = _sampled(N_E, 300, 6)
    terms = oracle_terms(d)
    E = energies_from_k(d.alpha, k[idx], q, t, mu)
    keep = far_from_poles(terms, d.n_int, E, w)
    idx, E = idx[keep], E[keep]
    ref, scale, dist, _ = reference_hubbard(d, k[idx], q, t, mu, w, beta, terms=terms)
    st = {}
    check(out[:, torch.from_numpy(idx).to(DEV)].cpu().numpy(), ref, scale, dist, label="full-size adjoint values",
          stats=st)
    print(f"adjoint step values: {st}", flush=True)
    cot = np.full((1, len(idx)), c)
    dE, _, _ = gradients(terms, d.n_int, E, w, beta, cot)
    dk, _, _ = momentum_gradients(d.alpha, k[idx], q, t, mu, dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, hubbard=(d.alpha, k[idx], q, t, mu))
    got = g_k[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    err = np.abs(got - dk.astype(np.float64)) / np.maximum(sc["k"], 1e-300)
    assert err.max() <= 1e-10, err.max()
