"""GPU parity: the HIP evaluator (called through the C ABI) against the oracle,
element by element, on seeded inputs.  Sizes span several blocks of lanes and
end in a ragged block."""
import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, order2_example,
                        random_self_energy, real_freqs, uniform_energies)

from parity import check, oracle_terms, reference, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"

# the packed (table-driven) and the specialized (generated) kernels
VARIANTS = pytest.mark.parametrize("variant", [amd.VARIANT_PACKED, amd.VARIANT_SPECIALIZED],
                                   ids=["packed", "specialized"])


def _terms(d, variant=amd.VARIANT_AUTO):
    t = amd.Terms.from_diagram(d)
    t.set_variant(variant)
    return t


def _gpu_eval(d, E, w, beta, e_reg=0.0, want_sum=False, terms=None, variant=amd.VARIANT_AUTO):
    t = terms if terms is not None else _terms(d, variant)
    Et = torch.from_numpy(np.ascontiguousarray(E)).to(DEV)
    wt = torch.from_numpy(np.asarray(w, dtype=np.complex128)).to(DEV)
    out, s = amd.evaluate(t, Et, wt, beta, e_reg, want_out=True, want_sum=want_sum)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (s.cpu().numpy() if s is not None else None)


@VARIANTS
def test_order2_paper_example(variant):
    """Sec. 5.1.3: the second-order integrand at energies uniform in (-8, 8),
    100 fermionic frequencies i(2j+1)pi at beta = 1 (fewer energy rows)."""
    d = order2_example()
    E = uniform_energies(1000, 3, seed=(1, 0), a=8.0)
    w = matsubara_freqs(100, 1.0)
    got, _ = _gpu_eval(d, E, w, 1.0, variant=variant)
    ref, scale, dist = reference(d, E, w, 1.0)
    check(got, ref, scale, dist, label="order2 paper example")


@pytest.mark.parametrize("order,i,beta,n_e", [
    (3, 0, 2.0, 1500), (3, 5, 10.0, 777), (4, 1, 5.0, 2049), (4, 6, 2.0, 1000),
    (5, 2, 5.0, 700), (6, 0, 5.0, 300),
])
@VARIANTS
def test_seeded_energy_path(order, i, beta, n_e, variant):
    d = random_self_energy(order, (0, order, i))
    E = uniform_energies(n_e, d.n_eps, seed=(2, order, i), a=4.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -6.0, 6.0, 0.05)])
    got, _ = _gpu_eval(d, E, w, beta, variant=variant)
    ref, scale, dist = reference(d, E, w, beta)
    check(got, ref, scale, dist, label=f"order {order} seed {i}")


@pytest.mark.parametrize("order,i", [(2, None), (4, 1), (4, 3), (5, 2)])
@VARIANTS
def test_hubbard_path(order, i, variant):
    d = order2_example() if i is None else random_self_energy(order, (0, order, i))
    beta, t, mu = 5.0, 1.0, 0.1
    k = k_samples(1300, d.n_int, seed=(3, order, 0 if i is None else i))
    q = np.array(DEFAULT_Q)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(3, -6.0, 6.0, 0.05)])
    T = _terms(d, variant)
    kt = torch.from_numpy(k).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    out, _ = amd.evaluate_hubbard(T, kt, q, t, mu, wt, beta)
    torch.cuda.synchronize()
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta)
    check(out.cpu().numpy(), ref, scale, dist, label=f"hubbard order {order}")


def test_row_sums_and_determinism():
    d = random_self_energy(4, (0, 4, 2))
    beta = 5.0
    E = uniform_energies(5000, d.n_eps, seed=7, a=4.0)
    w = matsubara_freqs(3, beta)
    T = amd.Terms.from_diagram(d)
    Et = torch.from_numpy(E).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    o1, s1 = amd.evaluate(T, Et, wt, beta, want_sum=True)
    o2, s2 = amd.evaluate(T, Et, wt, beta, want_sum=True)
    _, s3 = amd.evaluate(T, Et, wt, beta, want_out=False, want_sum=True)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2) and torch.equal(s1, s2) and torch.equal(s1, s3)
    ref, scale, dist = reference(d, E, w, beta)
    want = ref.sum(axis=1)
    err = np.abs(s1.cpu().numpy() - want) / scale.sum(axis=1)
    assert err.max() <= 1e-10
    # the row sum equals the sum of the returned rows
    np.testing.assert_allclose(s1.cpu().numpy(), o1.cpu().numpy().sum(axis=1), rtol=1e-12)


def test_strided_energies_bitwise_equal():
    d = random_self_energy(4, (0, 4, 3))
    beta = 2.0
    E = uniform_energies(999, d.n_eps, seed=8, a=4.0)
    w = matsubara_freqs(2, beta)
    T = amd.Terms.from_diagram(d)
    aos = torch.from_numpy(E).to(DEV)
    soa = torch.from_numpy(np.ascontiguousarray(E.T)).to(DEV).t()   # column-major view
    assert soa.stride() == (1, 999)
    wt = torch.from_numpy(w).to(DEV)
    o1, _ = amd.evaluate(T, aos, wt, beta)
    o2, _ = amd.evaluate(T, soa, wt, beta)
    # full frequency rows (internal slots zero-filled, Sec. 2.3) select the external slot
    full = torch.zeros((2, d.n_freq), dtype=torch.complex128, device=DEV)
    full[:, -1] = wt
    o3, _ = amd.evaluate(T, aos, full, beta)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2) and torch.equal(o1, o3)


@pytest.mark.parametrize("n_e", [0, 1, 63, 64, 65, 257])
def test_small_and_empty_batches(n_e):
    d = order2_example()
    beta = 5.0
    E = uniform_energies(max(n_e, 1), 3, seed=9, a=4.0)[:n_e]
    w = matsubara_freqs(2, beta)
    T = amd.Terms.from_diagram(d)
    Et = torch.from_numpy(np.ascontiguousarray(E)).to(DEV).reshape(n_e, 3)
    wt = torch.from_numpy(w).to(DEV)
    out, s = amd.evaluate(T, Et, wt, beta, want_sum=True)
    torch.cuda.synchronize()
    assert out.shape == (2, n_e)
    if n_e == 0:
        assert torch.all(s == 0)
        return
    ref, scale, dist = reference(d, E, w, beta)
    check(out.cpu().numpy(), ref, scale, dist, label=f"n_e={n_e}")


@VARIANTS
def test_regulator_on_bose_leaves(variant):
    d = order2_example()
    beta, e_reg = 5.0, 0.05
    E = uniform_energies(800, 3, seed=10, a=4.0)
    w = matsubara_freqs(2, beta)
    got, _ = _gpu_eval(d, E, w, beta, e_reg=e_reg, variant=variant)
    ref, scale, dist = reference(d, E, w, beta, e_reg=e_reg)
    check(got, ref, scale, dist, label="e_reg")


@VARIANTS
def test_bosonic_external_bubble(variant):
    alpha = np.array([[1, 0], [1, 1]])
    eps = np.eye(2, dtype=np.int8)
    from ami_inputs import Diagram
    d = Diagram(alpha=alpha.astype(np.int8), eps=eps, n_int=1,
                fermionic=np.array([1, 0], dtype=np.uint8))
    beta = 3.0
    E = uniform_energies(600, 2, seed=11, a=3.0)
    w = 2j * np.pi * np.arange(1, 5) / beta
    got, _ = _gpu_eval(d, E, w, beta, variant=variant)
    ref, scale, dist = reference(d, E, w, beta)
    check(got, ref, scale, dist, label="bubble")


def test_host_argument_checks():
    d = order2_example()
    T = amd.Terms.from_diagram(d)
    E = torch.zeros((10, 4), dtype=torch.float64, device=DEV)
    w = torch.zeros((1,), dtype=torch.complex128, device=DEV)
    with pytest.raises(amd.AmiError):
        amd.evaluate(T, E, w, 1.0)
    with pytest.raises(amd.AmiError):
        amd.evaluate(T, E[:, :3], w, -1.0)
    with pytest.raises(amd.AmiError):
        amd.evaluate(T, E[:, :3], w, 1.0, want_out=False, want_sum=False)


@VARIANTS
def test_full_size_sampled_order4_hubbard(variant):
    """The benchmark's launch: order-4 diagram, 10^6 momentum samples, one
    Matsubara frequency; 2000 sampled outputs checked one by one."""
    d = random_self_energy(4, (0, 4, 1))
    beta, t, mu = 5.0, 1.0, 0.0
    n_e = 1_000_000
    k = k_samples(n_e, d.n_int, seed=(4, 4, 1))
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    T = _terms(d, variant)
    out, s = amd.evaluate_hubbard(T, torch.from_numpy(k).to(DEV), q, t, mu,
                                  torch.from_numpy(w).to(DEV), beta, want_sum=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    idx = np.sort(np.random.default_rng(0).choice(n_e, 2000, replace=False))
    idx[-1] = n_e - 1
    terms = oracle_terms(d)
    ref, scale, dist, _ = reference_hubbard(d, k[idx], q, t, mu, w, beta, terms=terms)
    check(out[:, idx], ref, scale, dist, label="full size sampled")
    assert np.all(np.isfinite(out))
    np.testing.assert_allclose(s.cpu().numpy(), out.sum(axis=1), rtol=1e-9)
