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
    # forward and adjoint (both forms of its leaf-cotangent sweep), once
    assert len(list(tmp_path.glob("*.hsaco"))) == 3
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


def test_workspaces_on_several_streams():
    """Each stream has its own partial-sum workspace: calls that alternate
    between two streams give the same bits, and match the packed path (its
    own launch shape) to rounding."""
    d = random_self_energy(4, (0, 4, 1))
    T = amd.Terms.from_diagram(d)
    beta = 5.0
    q = np.array(DEFAULT_Q)
    k = torch.from_numpy(k_samples(70000, d.n_int, seed=52)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(3, beta)).to(DEV)
    gs = torch.tensor([1.0, 0.5j, -0.25], dtype=torch.complex128, device=DEV)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    res = []
    for rep in range(4):
        s = streams[rep % 2]
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            out_sum = torch.empty(3, dtype=torch.complex128, device=DEV)
            g = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs, out_sum=out_sum,
                                             stream=s)
            o, s2 = amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True, stream=s)
        torch.cuda.synchronize()
        assert amd.last_variant() == "specialized"
        res.append((out_sum, s2) + tuple(g[1:]))
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert torch.equal(x, y)
    # the adjoint's energies come from the sin/cos pair, the forward's from cos alone
    assert torch.allclose(res[0][0], res[0][1], rtol=1e-12, atol=0)
    T.set_variant(amd.VARIANT_PACKED)
    _, s3 = amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True)
    g3 = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs)
    torch.cuda.synchronize()
    assert torch.allclose(res[0][1], s3, rtol=1e-11, atol=0)
    for x, y in zip(res[0][2:], g3[1:]):
        assert torch.allclose(x, y, rtol=1e-9, atol=1e-12 * float(torch.abs(y).max()))


def test_step_replayed_as_a_graph():
    """Once a first call on a stream has loaded the kernels and sized the
    workspace, a value-and-gradient call allocates nothing and can be captured
    in a HIP graph; every replay, with eager work and synchronizations in
    between, gives the eager call's bits."""
    d = random_self_energy(4, (0, 4, 1))
    T = amd.Terms.from_diagram(d)
    beta = 5.0
    q = np.array(DEFAULT_Q)
    k = torch.from_numpy(k_samples(50000, d.n_int, seed=53)).to(DEV)
    w = torch.from_numpy(matsubara_freqs(1, beta)).to(DEV)
    gs = torch.ones(1, dtype=torch.complex128, device=DEV)
    out = torch.empty((1, 50000), dtype=torch.complex128, device=DEV)
    out_sum = torch.empty((1,), dtype=torch.complex128, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        grads = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs, out=out,
                                             out_sum=out_sum)
    torch.cuda.synchronize()
    ref = [out.clone(), out_sum.clone()] + [g.clone() for g in grads]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs, out=out, out_sum=out_sum,
                                     grads=grads)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device=DEV)
    for rep in range(4):
        out.fill_(float("nan"))
        out_sum.zero_()
        for x in grads:
            x.fill_(float("nan"))
        scratch.add_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip([out, out_sum] + list(grads), ref):
            assert torch.equal(x, y), rep
