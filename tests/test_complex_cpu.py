"""Complex energies in the library, on the CPU: the generated functions of
the complex-energy kernel (complex group sums over the diagram's own leaves
and denominators) and of its adjoint (complex leaf cotangents) compiled on
the host with the device leaf at a complex argument, compared with the
oracle's values and gradients; the host-side refusals."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from ami_inputs import complex_energies, matsubara_freqs, order2_example, random_self_energy, real_freqs
from oracle.evaluate import evaluate_terms, gradients, term_magnitudes

from parity import check, far_from_poles, gradient_scales, oracle_terms, pole_distance

amd = pytest.importorskip("paper_2311_17189_amd")

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [("o2", None), ("o3", (0, 3, 0)), ("o4", (0, 4, 1)), ("o5", (0, 5, 2))]


def _harness(src, tmp_path, name, driver="jit_check_complex.cpp"):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    body = "\n".join(l for l in src.splitlines()
                     if l.strip() not in ('#include "kargs.hpp"', '#include "jit_kernel.hpp"'))
    gen = tmp_path / f"{name}.inc"
    gen.write_text(body)
    exe = str(tmp_path / name)
    subprocess.run([cxx, "-O1", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(HERE, "cpu_math", "shim"),
                    f'-DAMI_GENERATED="{gen}"', os.path.join(HERE, "cpu_math", driver),
                    "-o", exe], check=True, capture_output=True, text=True)
    return exe


def _run(exe, beta, e_reg, w, E):
    lines = [f"{len(E)} {len(w)} {beta!r} {e_reg!r}",
             " ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in np.asarray(w).ravel())]
    for row in E:
        lines.append(" ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in row))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    out = np.array([[float(v) for v in l.split()] for l in res.stdout.strip().splitlines()])
    return (out[:, 0::2] + 1j * out[:, 1::2]).T


# two-pass complex sources: o4 52 terms, o6 560, and an order-6 topology of
# 2804 terms (above the one-pass size, where only these kernels serve)
TWO_PASS_CASES = [("o4", (0, 4, 1), 150), ("o6", (0, 6, 0), 40), ("o6big", (5, 6, 2), 12)]


@pytest.mark.parametrize("name,seed,n", TWO_PASS_CASES)
def test_generated_complex_two_pass_matches_oracle(name, seed, n, tmp_path):
    d = random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False, two_pass=True)
    assert "group_sums_c_store" in src and "group_accumulate_c" in src
    exe = _harness(src, tmp_path, name + "t", "jit_check_complex_two_pass.cpp")
    beta, e_reg = 4.0, 0.02
    E = complex_energies(3 * n, d.n_eps, seed=(93, d.n_int), a=3.0, eta=0.03)
    w = np.concatenate([matsubara_freqs(1, beta), real_freqs(1, 0.7, 0.7, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)][:n])
    got = _run(exe, beta, e_reg, w, E)
    ref = evaluate_terms(terms, d.n_int, E, w, beta, e_reg).astype(np.complex128)
    scale = term_magnitudes(terms, d.n_int, E, w, beta, e_reg).astype(np.float64)
    check(got, ref, scale, pole_distance(terms, d.n_int, E, w, e_reg), label=f"{name} complex two-pass")


@pytest.mark.parametrize("name,seed", CASES)
@pytest.mark.parametrize("e_reg", [0.0, 0.03])
@pytest.mark.parametrize("nested", ["0", "4"], ids=["term_products", "nested_sweep"])
def test_generated_complex_adjoint_matches_oracle(name, seed, e_reg, nested, tmp_path, monkeypatch):
    """The adjoint at complex energies in one pass: dL/dRe E + i dL/dIm E per
    sample, dL/dbeta and dL/dw summed, within 1e-10 of their rounding scales;
    the values formed on the way within the forward's bar."""
    monkeypatch.setenv("AMIGPU_JIT_NESTED_COTANGENTS", nested)
    d = order2_example() if seed is None else random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False)
    assert "leaf_cotangents_c" in src
    _check_complex_adjoint(d, _harness(src, tmp_path, name + "a", "jit_check_cadj.cpp"), e_reg, name)


# the adjoint at complex energies in passes: o4 52 terms, o5 196, o6 560
CADJ_PASS_CASES = [("o2", None, 0.0), ("o4", (0, 4, 1), 0.03), ("o5", (0, 5, 2), 0.0), ("o6", (0, 6, 0), 0.03)]


@pytest.mark.parametrize("name,seed,e_reg", CADJ_PASS_CASES)
def test_generated_complex_adjoint_passes_match_oracle(name, seed, e_reg, tmp_path):
    """The same through the three passes (complex group sums stored, the
    frequency pass, the leaf pass's complex reverse sweep)."""
    d = order2_example() if seed is None else random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False, two_pass=True)
    assert "cadj_freq_row" in src and "void cleaf_pass(" in src
    n = 120 if seed is None or seed[1] < 6 else 30
    _check_complex_adjoint(d, _harness(src, tmp_path, name + "ap", "jit_check_cadj_passes.cpp"), e_reg, name, n)


def _check_complex_adjoint(d, exe, e_reg, name, n=120):
    beta = 4.0
    E = complex_energies(n, d.n_eps, seed=(91, d.n_int), a=3.0, eta=0.05)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.4, 0.4, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    rng = np.random.default_rng(92)
    cot = rng.standard_normal((len(w), len(E))) + 1j * rng.standard_normal((len(w), len(E)))
    lines = [f"{len(E)} {len(w)} {beta!r} {e_reg!r}",
             " ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in w)]
    for s in range(len(E)):
        lines.append(" ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in E[s]) + " " +
                     " ".join(f"{float(c.real)!r} {float(c.imag)!r}" for c in cot[:, s]))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    out = np.array([[float(v) for v in l.split()] for l in res.stdout.strip().splitlines()])
    n_f, ne = len(w), d.n_eps
    vals = (out[:, 0:2 * n_f:2] + 1j * out[:, 1:2 * n_f:2]).T
    gE = out[:, 2 * n_f:2 * n_f + 2 * ne:2] + 1j * out[:, 2 * n_f + 1:2 * n_f + 2 * ne:2]
    gb = out[:, 2 * n_f + 2 * ne].sum()
    rest = out[:, 2 * n_f + 2 * ne + 1:]
    gw = (rest[:, 0::2] + 1j * rest[:, 1::2]).sum(axis=0)
    ref = evaluate_terms(terms, d.n_int, E, w, beta, e_reg).astype(np.complex128)
    scale = term_magnitudes(terms, d.n_int, E, w, beta, e_reg).astype(np.float64)
    check(vals, ref, scale, pole_distance(terms, d.n_int, E, w), label=f"{name} complex adjoint values")
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot, e_reg)
    sc = gradient_scales(terms, d.n_int, E, w, beta, cot, e_reg)
    assert np.max(np.abs(gE - dE.astype(np.complex128)) / np.maximum(sc["E"], 1e-300)) <= 1e-10
    assert abs(gb - float(db)) <= 1e-10 * sc["beta"]
    assert np.max(np.abs(gw - dw.astype(np.complex128).ravel())) <= 1e-10 * sc["w"]


@pytest.mark.parametrize("name,seed", CASES)
def test_generated_complex_values_match_oracle(name, seed, tmp_path):
    d = order2_example() if seed is None else random_self_energy(seed[1], seed)
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False)
    assert "group_sums_c" in src
    exe = _harness(src, tmp_path, name)
    beta, e_reg = 4.0, 0.0
    E = complex_energies(250, d.n_eps, seed=(90, d.n_int), a=3.0, eta=0.05)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(2, -2.0, 2.0, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    got = _run(exe, beta, e_reg, w, E)
    ref = evaluate_terms(terms, d.n_int, E, w, beta).astype(np.complex128)
    scale = term_magnitudes(terms, d.n_int, E, w, beta).astype(np.float64)
    check(got, ref, scale, pole_distance(terms, d.n_int, E, w), label=f"{name} complex energies")


def test_complex_source_omitted_for_taylor_leaves():
    alpha = np.array([[1, 0], [1, 0], [1, 1]])
    eps = np.array([[1, 0], [1, 0], [0, 1]])
    T = amd.Terms(alpha, eps, 1, [1, 0], multipole=True)
    assert "group_sums_c" not in T.source(momentum=False)
    assert "group_sums_c" not in amd.Terms.from_diagram(order2_example()).source(momentum=True)
