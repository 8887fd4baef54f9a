"""The run-time specialized kernels on the GPU beyond the parity tests that
run every variant: compilation ahead of use, the code-object cache across
handles, and the kernel timer the benchmark reads."""
import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy

from parity import check, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


def test_specialize_ahead_and_cache_across_handles(tmp_path, monkeypatch):
    monkeypatch.setenv("AMIGPU_CACHE_DIR", str(tmp_path))
    d = random_self_energy(4, (0, 4, 2))
    beta, t, mu = 5.0, 1.0, 0.0
    q = np.array(DEFAULT_Q)
    k = k_samples(3000, d.n_int, seed=(50, 4))
    w = matsubara_freqs(2, beta)
    kt, wt = torch.from_numpy(k).to(DEV), torch.from_numpy(w).to(DEV)
    outs = []
    for _ in range(2):
        T = amd.Terms.from_diagram(d)
        T.set_variant(amd.VARIANT_SPECIALIZED)
        T.specialize(momentum=True)               # compiles, or loads the cached code object
        o, s = amd.evaluate_hubbard(T, kt, q, t, mu, wt, beta, want_sum=True)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized"
        outs.append((o, s))
    assert len(list(tmp_path.glob("*.hsaco"))) == 2          # forward and adjoint, once
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    ref, scale, dist, _ = reference_hubbard(d, k, q, t, mu, w, beta)
    check(outs[0][0].cpu().numpy(), ref, scale, dist, label="cached specialized")


def test_kernel_timer_records_main_kernels():
    d = random_self_energy(3, (0, 3, 0))
    T = amd.Terms.from_diagram(d)
    beta = 5.0
    k = torch.from_numpy(k_samples(100000, d.n_int, seed=51)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(1, beta)).to(DEV)
    gs = torch.ones(1, dtype=torch.complex128, device=DEV)
    q = np.array(DEFAULT_Q)
    amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta)      # compile outside the timer
    amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs)
    torch.cuda.synchronize()
    amd.kernel_timer_start(2)
    for _ in range(3):                                            # the third is not recorded
        amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True)
    ms = amd.kernel_timer_stop()
    assert len(ms) == 2 and all(0.0 < v < 1000.0 for v in ms)
    with pytest.raises(amd.AmiError):
        amd.kernel_timer_stop()                                   # not running any more
