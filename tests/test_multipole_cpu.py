"""Poles of higher order (Eq. (5)) in the library, on the CPU: the construction
with AMI_MULTIPOLE against the oracle's term stream, bit for bit (including the
extended stream of terms with unequal denominator counts), the error paths,
and the generated straight-line functions (Taylor-coefficient leaves and their
slopes, groups with unequal denominator lists) compiled on the host and
compared with the oracle's values and analytic gradients."""
import numpy as np
import pytest

from ami_inputs import matsubara_freqs, random_self_energy, real_freqs, uniform_energies
from oracle.construct import canonical, construct, serialize
from oracle.evaluate import evaluate_terms, gradients, term_magnitudes

from parity import check, far_from_poles, gradient_scales, pole_distance
from multipole_cases import CASES, DOUBLE, repeated_line  # noqa: F401

amd = pytest.importorskip("paper_2311_17189_amd")

from test_specialized_cpu import _harness, _run  # noqa: E402

def _oracle(case):
    alpha, eps, n_int, ferm = case
    return canonical(construct(alpha, eps, n_int, ferm, multipole=True))


@pytest.mark.parametrize("name", list(CASES))
def test_multipole_stream_matches_oracle(name):
    alpha, eps, n_int, ferm = CASES[name]
    T = amd.Terms(alpha, eps, n_int, ferm, multipole=True)
    terms = _oracle(CASES[name])
    want = np.array(serialize(terms, n_int, eps.shape[1], alpha.shape[1]), dtype=np.int32)
    got = T.canonical()
    assert np.array_equal(got, want)
    inf = T.info()
    assert inf["T"] == len(terms) and inf["n_g"] == alpha.shape[0]
    assert inf["uniform"] == 0 and inf["packable"] == 0
    assert any(abs(c) > 1 for _, lv, _ in terms for c, _ in lv)
    a2, e2, f2 = T.labels()
    assert np.array_equal(a2, alpha) and np.array_equal(e2, eps) and list(f2) == list(ferm)


def test_multipole_errors_and_simple_poles_unchanged():
    alpha, eps, n_int, ferm = DOUBLE
    with pytest.raises(amd.AmiError) as e:
        amd.Terms(alpha, eps, n_int, ferm)
    assert e.value.code == -3
    with pytest.raises(amd.AmiError) as e:
        amd.Terms(alpha, eps, n_int, ferm, factorize=True, multipole=True)
    assert e.value.code == -7
    for order, i in ((2, 0), (3, 1), (4, 1)):
        d = random_self_energy(order, (0, order, i))
        a = amd.Terms.from_diagram(d)
        b = amd.Terms.from_diagram(d, multipole=True)
        assert np.array_equal(a.canonical(), b.canonical())
        assert b.info()["uniform"] == 1


def _multipole_inputs(name, n=200):
    alpha, eps, n_int, ferm = CASES[name]
    beta = 4.0
    E = uniform_energies(n, eps.shape[1], seed=(44, n_int, alpha.shape[0]), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.6, 0.6, 0.05)])
    if not ferm[-1]:
        w = np.concatenate([2j * np.pi * np.arange(1, 3) / beta, real_freqs(1, 0.6, 0.6, 0.05)])
    terms = _oracle(CASES[name])
    E = np.ascontiguousarray(E[far_from_poles(terms, n_int, E, w)])
    rng = np.random.default_rng(48)
    cot = rng.standard_normal((len(w), len(E))) + 1j * rng.standard_normal((len(w), len(E)))
    return terms, beta, E, w, cot


def _check_multipole(name, exe, label):
    alpha, eps, n_int, ferm = CASES[name]
    terms, beta, E, w, cot = _multipole_inputs(name)
    vals, gE, gb, _, _, gw = _run(exe, eps.shape[1], len(w), beta, 0.0, 1.0, 0.0, np.zeros(2), w[:, None], E, cot)
    ref = evaluate_terms(terms, n_int, E, w, beta).astype(np.complex128)
    scale = term_magnitudes(terms, n_int, E, w, beta).astype(np.float64)
    check(vals, ref, scale, pole_distance(terms, n_int, E, w), label=f"{name} multipole values ({label})")
    # the adjoint: dT_j/dx = (j + 1) T_(j+1) and dT_j/dbeta = (j T_j + x dT_j/dx) / beta
    # for the Taylor-coefficient leaves, powers of denominators as repeated factors
    dE, db, dw = gradients(terms, n_int, E, w, beta, cot)
    sc = gradient_scales(terms, n_int, E, w, beta, cot)
    assert np.max(np.abs(gE - dE.astype(np.float64)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(gb - float(db)) <= 1e-10 * sc["beta"]
    if alpha.shape[1] > n_int:
        assert np.max(np.abs(gw - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nested", ["0", "4"], ids=["term_products", "nested_sweep"])
def test_generated_multipole_values_and_gradients_match_oracle(name, nested, tmp_path, monkeypatch):
    monkeypatch.setenv("AMIGPU_JIT_NESTED_COTANGENTS", nested)
    T = amd.Terms(*CASES[name], multipole=True)
    src = T.source(momentum=False)
    assert "taylor_slopes" in src and "constexpr bool kTaylor = true;" in src
    _check_multipole(name, _harness(src, tmp_path, name), "one pass")


@pytest.mark.parametrize("name", list(CASES))
def test_generated_multipole_adjoint_passes_match_oracle(name, tmp_path):
    T = amd.Terms(*CASES[name], multipole=True)
    src = T.source(momentum=False, two_pass=True)
    assert "void leaf_pass(" in src and "DB0" in src
    _check_multipole(name, _harness(src, tmp_path, name + "p", "jit_check_adj_passes.cpp"), "passes")


def test_multipole_source_has_adjoint_not_complex(tmp_path, monkeypatch):
    """The generated source of a multipole solution holds the forward kernel
    and the adjoint (Taylor-coefficient leaves with their slopes), not the
    complex-energy kernel; amiTermsSpecialize compiles those (the adjoint in
    both forms of its leaf-cotangent sweep; here, with no device, it then
    stops at the device query)."""
    monkeypatch.setenv("AMIGPU_CACHE_DIR", str(tmp_path))
    T = amd.Terms(*DOUBLE, multipole=True)
    src = T.source(momentum=False)
    assert "taylor_leaves" in src and "#define AMI_JIT_KERNELS 3\n" in src
    with pytest.raises(amd.AmiError) as e:
        T.specialize(momentum=False)
    assert e.value.code == -5 and "hipGetDevice" in str(e.value)
    # the forward, and the adjoint in both forms of its leaf-cotangent sweep
    assert len([p for p in tmp_path.iterdir() if p.name.endswith(".hsaco")]) == 3


@pytest.mark.parametrize("name", list(CASES))
def test_structure_of_the_extended_stream(name):
    """The measurement code reads the extended stream (unequal denominator
    counts) into the same distinct leaves, denominators and groups as the
    library's tables."""
    from paper_2311_17189_amd import roofline as rl
    T = amd.Terms(*CASES[name], multipole=True)
    st = rl.structure_from_canonical(T.canonical())
    inf = T.info()
    assert (st.T, len(st.leaves), len(st.dens), len(st.groups)) == (inf["T"], inf["L"], inf["D"], inf["G"])
    assert sum(c for c, _ in st.groups) == st.T
    assert any(abs(c) > 1 for c, _ in st.leaves)
