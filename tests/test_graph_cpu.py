"""Feynman-graph input (Sec. 2.5) on the CPU: the library's reader and
labeller.  A diagram's integrand depends only on its graph and the energies
of its propagators, not on which loop frequencies label it, so the library's
labels for a generated graph must give the oracle the same values as the
generator's own labels, line by line."""
import numpy as np
import pytest

from ami_inputs import matsubara_freqs, random_self_energy, real_freqs, uniform_energies
from oracle.construct import canonical, construct
from oracle.evaluate import evaluate_terms, term_magnitudes

amd = pytest.importorskip("paper_2311_17189_amd")


def _values(alpha, eps, n_int, fermionic, E, w, beta):
    terms = canonical(construct(alpha, eps, n_int, fermionic))
    return (evaluate_terms(terms, n_int, E, w, beta).astype(np.complex128),
            term_magnitudes(terms, n_int, E, w, beta).astype(np.float64))


@pytest.mark.parametrize("order,i", [(2, 0), (3, 1), (4, 1), (4, 5), (5, 2)])
def test_graph_labels_give_the_generator_values(order, i):
    d = random_self_energy(order, (0, order, i))
    T = amd.Terms.from_graph(d.graph)
    alpha, eps, ferm = T.labels()
    n_int = T.info()["n_int"]
    assert n_int == order and alpha.shape == d.alpha.shape
    assert np.array_equal(eps, np.eye(d.n_g, dtype=np.int8)) and np.all(ferm == 1)
    assert set(np.unique(alpha)) <= {-1, 0, 1}
    # the loop lines carry unit labels, and every summed frequency appears
    assert np.all(np.count_nonzero(alpha[:, :n_int], axis=0) >= 1)
    beta = 3.0
    E = uniform_energies(400, d.n_g, seed=(70, order, i), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.4, 0.4, 0.05)])
    got, sc = _values(alpha, eps, n_int, ferm, E, w, beta)
    want, sc2 = _values(d.alpha, d.eps, d.n_int, d.fermionic, E, w, beta)
    assert np.max(np.abs(got - want) / np.maximum(sc, sc2)) <= 1e-12


def test_bosonic_external_bubble_graph():
    """Two fermionic lines between two vertices and no bosonic line: the
    external frequency is bosonic, entering at vertex 0 and leaving at 1."""
    T = amd.Terms.from_graph([[0, 1, 1, 0], [1, 0, 1, 0]])
    alpha, eps, ferm = T.labels()
    assert alpha.tolist() == [[1, 1], [1, 0]] and ferm.tolist() == [1, 0]
    beta = 2.0
    E = uniform_energies(300, 2, seed=71, a=3.0)
    w = 2j * np.pi * np.arange(1, 4) / beta
    got, sc = _values(alpha, eps, 1, ferm, E, w, beta)
    # the bubble (1/beta) sum 1/((i nu + E_a)(i nu + i Omega + E_b)) = [f(-E_a) - f(-E_b)] / (i Omega + E_b - E_a)
    # with line 1 (label nu) = E_a and line 0 (label nu + Omega) = E_b
    fa = 1.0 / (np.exp(-beta * E[:, 1]) + 1.0)
    fb = 1.0 / (np.exp(-beta * E[:, 0]) + 1.0)
    closed = (fa - fb)[None, :] / (w[:, None] + E[None, :, 0] - E[None, :, 1])
    assert np.max(np.abs(got - closed) / np.maximum(sc, 1e-300)) <= 1e-12


def test_read_graph_file_and_errors(tmp_path):
    d = random_self_energy(3, (0, 3, 2))
    p = tmp_path / "se3.graph"
    p.write_text("# order-3 self-energy\n\n" + "\n".join(" ".join(str(x) for x in r) for r in d.graph) +
                 "  # last line\n")
    e = amd.read_graph(str(p))
    assert e.tolist() == [list(r) for r in d.graph]
    T = amd.Terms.from_graph_file(str(p))
    assert np.array_equal(T.canonical(), amd.Terms.from_graph(d.graph).canonical())
    bad = tmp_path / "bad.graph"
    bad.write_text("0 1 1\n")
    with pytest.raises(amd.AmiError):
        amd.read_graph(str(bad))
    bad.write_text("0 1 2 0\n")
    with pytest.raises(amd.AmiError):
        amd.read_graph(str(bad))
    with pytest.raises(amd.AmiError):
        amd.read_graph(str(tmp_path / "missing.graph"))
    with pytest.raises(amd.AmiError):      # two vertices without an incoming fermionic line
        amd.Terms.from_graph([[0, 1, 1, 0], [2, 1, 1, 0], [1, 3, 1, 0]])
    with pytest.raises(amd.AmiError):      # disconnected
        amd.Terms.from_graph([[0, 1, 1, 0], [1, 0, 1, 0], [2, 3, 1, 0], [3, 2, 1, 0]])
    with pytest.raises(amd.AmiError):      # vertices with no fermionic line
        amd.Terms.from_graph([[0, 1, 1, 0], [1, 0, 1, 0], [2, 3, 0, 0], [3, 2, 0, 0], [0, 2, 0, 0]])
