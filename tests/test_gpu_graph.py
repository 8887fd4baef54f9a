"""Feynman-graph input (Sec. 2.5) through to the GPU: a 4-column graph file is
read and labelled by the library (amiReadGraph, amiConstructGraph), and the
solution it builds is evaluated by the HIP kernels.  On the energy input (one
energy per line) the integrand depends only on the graph, so the GPU values
must equal the oracle's on the generator's own labels; on the momentum input
the oracle takes the library's labels (the loop momenta follow the labels)."""
import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy, real_freqs,
                        uniform_energies)
from oracle.construct import canonical, construct

from parity import check, reference, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


def _graph_file(tmp_path, d, name):
    p = tmp_path / f"{name}.graph"
    p.write_text("# source target B/F spin\n" + "\n".join(" ".join(str(x) for x in r) for r in d.graph) + "\n")
    return str(p)


@pytest.mark.parametrize("order,i", [(2, 0), (3, 1), (4, 1), (5, 2)])
def test_graph_file_energy_path_matches_generator_labels(order, i, tmp_path):
    d = random_self_energy(order, (0, order, i))
    T = amd.Terms.from_graph_file(_graph_file(tmp_path, d, f"se{order}_{i}"))
    beta = 4.0
    E = uniform_energies(2000 + 37 * order, d.n_g, seed=(72, order, i), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -2.0, 2.0, 0.05)])
    out, s = amd.evaluate(T, torch.from_numpy(E).to(DEV), torch.from_numpy(w).to(DEV), beta, want_sum=True)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    # the oracle's construction of the library's labels: the same term list,
    # so the full parity bar (plain relative error included) applies
    alpha, eps, ferm = T.labels()
    lab = type(d)(alpha=alpha, eps=eps, n_int=T.info()["n_int"], fermionic=ferm)
    ref, scale, dist = reference(lab, E, w, beta)
    check(got, ref, scale, dist, label=f"graph file, order {order}")
    # the oracle's construction from the generator's own labels of the same
    # graph: another term list of the same integrand, whose rounding differs,
    # so the bar is relative to the larger of the two term-magnitude sums
    ref2, scale2, dist2 = reference(d, E, w, beta)
    check(got, ref2, np.maximum(scale, scale2), np.minimum(dist, dist2), cond_max=0.0,
          label=f"graph file vs generator labels, order {order}")
    np.testing.assert_allclose(s.cpu().numpy(), got.sum(axis=1), rtol=1e-11, atol=1e-12 * scale.sum())


@pytest.mark.parametrize("order,i", [(3, 1), (4, 5)])
def test_graph_file_momentum_path_and_adjoint(order, i, tmp_path):
    d = random_self_energy(order, (0, order, i))
    T = amd.Terms.from_graph_file(_graph_file(tmp_path, d, f"se{order}_{i}"))
    alpha, eps, ferm = T.labels()
    n_int = T.info()["n_int"]
    lab = type(d)(alpha=alpha, eps=eps, n_int=n_int, fermionic=ferm)
    # the library's term list is the oracle's construction of the same labels, bit for bit
    from oracle.construct import serialize
    terms = canonical(construct(alpha, eps, n_int, ferm))
    assert np.array_equal(T.canonical(), np.array(serialize(terms, n_int, eps.shape[1], alpha.shape[1]),
                                                  dtype=np.int32))
    beta, t, mu = 5.0, 1.0, 0.0
    q = np.array(DEFAULT_Q)
    k = k_samples(3000, n_int, seed=(73, order, i))
    w = matsubara_freqs(1, beta)
    kt = torch.from_numpy(k).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    out, _ = amd.evaluate_hubbard(T, kt, q, t, mu, wt, beta)
    torch.cuda.synchronize()
    ref, scale, dist, _ = reference_hubbard(lab, k, q, t, mu, w, beta, terms=terms)
    check(out.cpu().numpy(), ref, scale, dist, label=f"graph file momenta, order {order}")
    # the adjoint step of the graph-built handle: its values equal the forward's
    o2 = torch.empty_like(out)
    amd.evaluate_hubbard_adjoint(T, kt, q, t, mu, wt, beta, grad_sum=torch.ones(1, dtype=torch.complex128,
                                                                                  device=DEV), out=o2)
    torch.cuda.synchronize()
    check(o2.cpu().numpy(), ref, scale, dist, label=f"graph file adjoint values, order {order}")
