"""The allocation-free adjoint entry point (amiEvaluateHubbardAdjointNoAlloc)
against amiEvaluateHubbardAdjoint, through the C ABI: the same kernels on the
same inputs, so every output must be equal bit for bit, on two calls in a row
(the second with fewer samples, so the scratch holds the first call's partial
sums when the second starts); the values also against the oracle."""
import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy, real_freqs

from parity import check, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"
BETA, T_HOP, MU = 5.0, 1.0, 0.0


def _inputs(d, n_e, n_f, seed):
    k = k_samples(n_e, d.n_int, seed=seed)
    w = np.concatenate([matsubara_freqs(n_f - 1, BETA), real_freqs(1, -1.0, -1.0, 0.05)])
    rng = np.random.default_rng(seed)
    cot = rng.standard_normal((n_f, n_e)) + 1j * rng.standard_normal((n_f, n_e))
    cot_sum = rng.standard_normal(n_f) + 1j * rng.standard_normal(n_f)
    return k, w, cot, cot_sum


def _run(fn, T, k, w, cot, cot_sum):
    n_f, n_e = cot.shape
    out = torch.empty((n_f, n_e), dtype=torch.complex128, device=DEV)
    out_sum = torch.empty((n_f,), dtype=torch.complex128, device=DEV)
    g = fn(T, torch.from_numpy(k).to(DEV), DEFAULT_Q, T_HOP, MU, torch.from_numpy(w).to(DEV), BETA,
           grad_out=torch.from_numpy(cot).to(DEV), grad_sum=torch.from_numpy(cot_sum).to(DEV),
           out=out, out_sum=out_sum)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in g] + [out.cpu().numpy(), out_sum.cpu().numpy()]


@pytest.mark.parametrize("order,i,variant", [(4, 1, "specialized"), (5, 0, "specialized passes"),
                                             (3, 1, "specialized")])
def test_no_alloc_matches_the_allocating_entry(order, i, variant):
    d = random_self_energy(order, (0, order, i))
    T = amd.Terms.from_diagram(d)
    T.upload()
    T.specialize(True)
    for n_e, n_f, seed in [(5000, 2, (60, order, 0)), (777, 2, (60, order, 1))]:
        k, w, cot, cot_sum = _inputs(d, n_e, n_f, seed)
        print(f"no-alloc order {order} n_e {n_e}", flush=True)
        got = _run(amd.evaluate_hubbard_adjoint_no_alloc, T, k, w, cot, cot_sum)
        assert (variant in amd.last_variant()), amd.last_variant()
        want = _run(amd.evaluate_hubbard_adjoint, T, k, w, cot, cot_sum)
        for name, a, b in zip(["grad_k", "grad_mu", "grad_t", "grad_beta", "grad_freqs", "out", "out_sum"],
                              got, want):
            assert np.array_equal(a, b), f"{name} differs from amiEvaluateHubbardAdjoint (n_e {n_e})"
        ref, scale, dist, _ = reference_hubbard(d, k, np.array(DEFAULT_Q), T_HOP, MU, w, BETA)
        check(got[5], ref, scale, dist, label=f"no-alloc values, order {order}, n_e {n_e}")


def test_no_alloc_preconditions_and_limits():
    d = random_self_energy(4, (0, 4, 1))
    k, w, cot, cot_sum = _inputs(d, 300, 2, (61, 4, 0))
    T = amd.Terms.from_diagram(d)
    with pytest.raises(amd.AmiError, match="amiTermsUpload"):
        _run(amd.evaluate_hubbard_adjoint_no_alloc, T, k, w, cot, cot_sum)
    T.upload()
    with pytest.raises(amd.AmiError, match="amiTermsSpecialize"):
        _run(amd.evaluate_hubbard_adjoint_no_alloc, T, k, w, cot, cot_sum)
    T.specialize(True)
    # partial sums beyond the scratch: refused on the host before any launch
    n_e, n_f = 100000, 1000      # about 100 MB of partial sums
    kk = torch.zeros((n_e, 2 * d.n_int), dtype=torch.float64, device=DEV)
    ww = torch.from_numpy(matsubara_freqs(n_f, BETA)).to(DEV)
    gs = torch.zeros((n_f,), dtype=torch.complex128, device=DEV)
    with pytest.raises(amd.AmiError, match="scratch"):
        amd.evaluate_hubbard_adjoint_no_alloc(T, kk, DEFAULT_Q, T_HOP, MU, ww, BETA, grad_sum=gs)
    # no samples: zero sums
    k0 = torch.zeros((0, 2 * d.n_int), dtype=torch.float64, device=DEV)
    g = amd.evaluate_hubbard_adjoint_no_alloc(T, k0, DEFAULT_Q, T_HOP, MU, ww[:2], BETA, grad_sum=gs[:2])
    torch.cuda.synchronize()
    assert all(float(x) == 0.0 for x in g[1:4])
    assert not g[4].abs().any()
