"""The run-time specialized evaluator on the CPU: its generated source (the
diagram's straight-line functions, written by the library from its tables) is
compiled with the host compiler and driven one sample at a time through the
kernels' steps (tests/cpu_math/jit_check.cpp); values and every gradient are
compared with the oracle.  The same source is compiled for gfx950 with hipRTC
by the library itself (no device is needed for that)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, order2_example, random_self_energy,
                        real_freqs, uniform_energies)
from oracle.evaluate import energies_from_k, gradients, momentum_gradients

from parity import check, far_from_poles, gradient_scales, oracle_terms, reference

amd = pytest.importorskip("paper_2311_17189_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


def _harness(src: str, tmp_path, name: str, driver: str = "jit_check.cpp") -> str:
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    body = "\n".join(l for l in src.splitlines()
                     if l.strip() not in ('#include "kargs.hpp"', '#include "jit_kernel.hpp"'))
    gen = tmp_path / f"{name}.inc"
    gen.write_text(body)
    exe = str(tmp_path / name)
    subprocess.run([cxx, "-O1", "-std=c++17", "-ffp-contract=off",
                    "-I", os.path.join(HERE, "cpu_math", "shim"),
                    f'-DAMI_GENERATED="{gen}"', os.path.join(HERE, "cpu_math", driver),
                    "-o", exe], check=True, capture_output=True, text=True)
    return exe


def _run(exe, rows, n_f, beta, e_reg, t, mu, q, w, inputs, cot):
    n_ext = w.shape[1]
    lines = [f"{len(inputs)} {n_f} {beta!r} {e_reg!r} {t!r} {mu!r}",
             " ".join(repr(float(v)) for v in np.asarray(q).ravel()[:2 * n_ext])]
    lines.append(" ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in w.ravel()))
    for s in range(len(inputs)):
        lines.append(" ".join(repr(float(v)) for v in inputs[s]) + " " +
                     " ".join(f"{float(c.real)!r} {float(c.imag)!r}" for c in cot[:, s]))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    out = np.array([[float(v) for v in l.split()] for l in res.stdout.strip().splitlines()])
    assert out.shape[0] == len(inputs)
    vals = out[:, 0:2 * n_f:2] + 1j * out[:, 1:2 * n_f:2]
    g_in = out[:, 2 * n_f:2 * n_f + rows]
    rest = out[:, 2 * n_f + rows:]
    gw = rest[:, 3::2] + 1j * rest[:, 4::2]
    return vals.T, g_in, rest[:, 0].sum(), rest[:, 1].sum(), rest[:, 2].sum(), gw.sum(axis=0).reshape(n_f, n_ext)


# o5: 196 terms, above the adjoint's automatic size, so the values come from
# the nested sum over groups (groups_combine)
CASES = [("o2", None), ("o3", (0, 3, 0)), ("o4", (0, 4, 1)), ("o4b", (0, 4, 3)), ("o5", (0, 5, 2))]


@pytest.mark.parametrize("name,seed", CASES)
@pytest.mark.parametrize("nested", ["0", "4"], ids=["term_products", "nested_sweep"])
def test_generated_energy_kernels_match_oracle(name, seed, nested, tmp_path, monkeypatch):
    """Values and gradients of the generated one-pass functions, with the
    leaf cotangents from per-term products and from the reverse sweep of the
    nested group sums (parts of four terms)."""
    monkeypatch.setenv("AMIGPU_JIT_NESTED_COTANGENTS", nested)
    d = order2_example() if seed is None else random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    exe = _harness(T.source(momentum=False), tmp_path, name)
    beta, e_reg = 5.0, 0.0
    E = uniform_energies(200, d.n_eps, seed=(40, d.n_int), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.7, 0.7, 0.05)])
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, E, w)
    E = np.ascontiguousarray(E[keep])
    rng = np.random.default_rng(41)
    cot = rng.standard_normal((len(w), len(E))) + 1j * rng.standard_normal((len(w), len(E)))
    vals, gE, gb, _, _, gw = _run(exe, d.n_eps, len(w), beta, e_reg, 1.0, 0.0, np.zeros(2),
                                  w[:, None], E, cot)
    ref, scale, dist = reference(d, E, w, beta)
    check(vals, ref, scale, dist, label=f"{name} values")
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot)
    assert np.max(np.abs(gE - dE.astype(np.float64)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(gb - float(db)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(gw - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


@pytest.mark.parametrize("name,seed", CASES)
@pytest.mark.parametrize("nested", ["0", "4"], ids=["term_products", "nested_sweep"])
def test_generated_momentum_kernels_match_oracle(name, seed, nested, tmp_path, monkeypatch):
    monkeypatch.setenv("AMIGPU_JIT_NESTED_COTANGENTS", nested)
    d = order2_example() if seed is None else random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    exe = _harness(T.source(momentum=True), tmp_path, name + "k")
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    k = k_samples(300, d.n_int, seed=(42, d.n_int))
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu), w)
    k = np.ascontiguousarray(k[keep])
    rng = np.random.default_rng(43)
    cot = rng.standard_normal((1, len(k))) + 1j * rng.standard_normal((1, len(k)))
    vals, gk, gb, gmu, gt, gw = _run(exe, 2 * d.n_int, 1, beta, 0.0, t, mu, q, w[:, None], k, cot)
    E = energies_from_k(d.alpha, k, q, t, mu)
    ref, scale, dist = reference(d, E, w, beta)
    check(vals, ref, scale, dist, label=f"{name} momentum values")
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, hubbard=(d.alpha, k, q, t, mu))
    assert np.max(np.abs(gk - dk.astype(np.float64)) / np.maximum(sc["k"], 1e-300)) <= 1e-10
    for got, ref_, key in ((gb, db, "beta"), (gmu, dmu, "mu"), (gt, dt, "t")):
        assert abs(got - float(ref_)) <= 1e-10 * sc[key], key
    assert np.max(np.abs(gw - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


# the adjoint of large solutions in passes (its functions are in the two-pass
# source of any solution): o4 52 terms, o5 196, o6 560
PASS_CASES = [("o4", (0, 4, 1), 120), ("o5", (0, 5, 2), 80), ("o6", (0, 6, 0), 30)]


@pytest.mark.parametrize("name,seed,n", PASS_CASES)
def test_adjoint_passes_energy_input_match_oracle(name, seed, n, tmp_path):
    d = random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False, two_pass=True)
    assert "adj_freq_row" in src and "void leaf_pass(" in src
    exe = _harness(src, tmp_path, name + "p", "jit_check_adj_passes.cpp")
    beta = 5.0
    E = uniform_energies(n, d.n_eps, seed=(44, d.n_int), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, -0.3, -0.3, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    rng = np.random.default_rng(45)
    cot = rng.standard_normal((len(w), len(E))) + 1j * rng.standard_normal((len(w), len(E)))
    vals, gE, gb, _, _, gw = _run(exe, d.n_eps, len(w), beta, 0.0, 1.0, 0.0, np.zeros(2), w[:, None], E, cot)
    ref, scale, dist = reference(d, E, w, beta)
    check(vals, ref, scale, dist, label=f"{name} values (passes)")
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot)
    assert np.max(np.abs(gE - dE.astype(np.float64)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(gb - float(db)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(gw - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


@pytest.mark.parametrize("name,seed,n", PASS_CASES)
def test_adjoint_passes_momentum_input_match_oracle(name, seed, n, tmp_path):
    d = random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    exe = _harness(T.source(momentum=True, two_pass=True), tmp_path, name + "pk", "jit_check_adj_passes.cpp")
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(1, beta)
    k = k_samples(2 * n, d.n_int, seed=(46, d.n_int))
    terms = oracle_terms(d)
    keep = far_from_poles(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu), w)
    k = np.ascontiguousarray(k[keep][:n])
    rng = np.random.default_rng(47)
    cot = rng.standard_normal((1, len(k))) + 1j * rng.standard_normal((1, len(k)))
    vals, gk, gb, gmu, gt, gw = _run(exe, 2 * d.n_int, 1, beta, 0.0, t, mu, q, w[:, None], k, cot)
    E = energies_from_k(d.alpha, k, q, t, mu)
    ref, scale, dist = reference(d, E, w, beta)
    check(vals, ref, scale, dist, label=f"{name} momentum values (passes)")
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, hubbard=(d.alpha, k, q, t, mu))
    assert np.max(np.abs(gk - dk.astype(np.float64)) / np.maximum(sc["k"], 1e-300)) <= 1e-10
    for got, ref_, key in ((gb, db, "beta"), (gmu, dmu, "mu"), (gt, dt, "t")):
        assert abs(got - float(ref_)) <= 1e-10 * sc[key], key
    assert np.max(np.abs(gw - dw.astype(np.complex128))) <= 1e-10 * sc["w"]


def test_source_limits_and_errors():
    d = order2_example()
    src = amd.Terms.from_diagram(d).source(momentum=True)
    assert "constexpr int NE = 3, NI = 2, NG = 3, NX = 1;" in src
    assert "constexpr int L = 4, D = 1, G = 1;" in src
    big = amd.Terms.from_diagram(random_self_energy(6, (5, 6, 0)))
    assert big.info()["T"] > 1024
    with pytest.raises(amd.AmiError) as e:
        big.source()
    assert e.value.code == -7


@pytest.mark.parametrize("momentum,kernels", [(True, (1, 2)), (False, (1, 2, 8, 256))])
def test_hiprtc_compiles_the_generated_source(tmp_path, monkeypatch, momentum, kernels):
    """amiTermsSpecialize compiles every kernel of the input for gfx950 before
    it needs a device (the complex-energy forward and adjoint too, for the
    energy input);
    here (no GPU) it then stops at the device query, leaving the code objects
    and their sources in the disk cache.  A second handle finds them there."""
    monkeypatch.setenv("AMIGPU_CACHE_DIR", str(tmp_path))
    d = random_self_energy(3, (0, 3, 0))
    for _ in range(2):
        T = amd.Terms.from_diagram(d)
        try:
            T.specialize(momentum=momentum)
        except amd.AmiError as e:
            assert e.code == -5 and "hipGetDevice" in str(e), str(e)
    srcs = sorted(p for p in tmp_path.iterdir() if p.name.endswith(".hip"))
    objs = sorted(p for p in tmp_path.iterdir() if p.name.endswith(".hsaco"))
    # one code object per kernel (forward 1, adjoint 2, complex-energy forward
    # 8 and adjoint 256), the one-pass adjoints in both forms of their
    # leaf-cotangent sweep
    two_forms = tuple(k for k in kernels if k in (2, 256))
    assert len(srcs) == len(objs) == len(kernels) + len(two_forms)
    for p in objs:
        assert p.stat().st_size > 1000
    found = sorted(k for p in srcs for k in kernels if f"#define AMI_JIT_KERNELS {k}\n" in p.read_text())
    assert found == sorted(kernels + two_forms)


def test_persistent_batch_module_compiles(tmp_path, monkeypatch):
    """The source of one persistent batch module -- several diagrams' generated
    functions, each in a namespace of its own with the tile functions, one
    solution in two passes, and the persistent kernels -- compiles for gfx950
    with hipRTC (no device needed)."""
    monkeypatch.setenv("AMIGPU_CACHE_DIR", str(tmp_path))
    ds = [random_self_energy(6, (0, 6, 0)), order2_example(), random_self_energy(3, (0, 3, 1)),
          random_self_energy(4, (0, 4, 1))]
    ts = [amd.Terms.from_diagram(d) for d in ds]
    src = amd.batch_source(ts, [16, 16, 16, 1], momentum=True, compile=True)
    for j in range(len(ds)):
        assert f"#define amijit amijit_b{j}" in src
    assert "ami_batch_p1" in src and "ami_batch_p2" in src         # order 6 (first): two passes
    assert "amijit_b3::fwd_tile<true, true>" in src                 # one frequency row
    assert "amijit_b1::fwd_tile<true, false>" in src
    objs = [p for p in tmp_path.iterdir() if p.name.endswith(".hsaco")]
    assert len(objs) == 1 and objs[0].stat().st_size > 10000
