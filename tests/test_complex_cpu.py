"""Complex energies in the library, on the CPU: the generated functions of
the complex-energy kernel (complex group sums over the diagram's own leaves
and denominators) compiled on the host with the device leaf at a complex
argument, compared with the oracle's values; the host-side refusals."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from ami_inputs import complex_energies, matsubara_freqs, order2_example, random_self_energy, real_freqs
from oracle.evaluate import evaluate_terms, term_magnitudes

from parity import check, far_from_poles, oracle_terms, pole_distance

amd = pytest.importorskip("paper_2311_17189_amd")

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [("o2", None), ("o3", (0, 3, 0)), ("o4", (0, 4, 1)), ("o5", (0, 5, 2))]


def _harness(src, tmp_path, name):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    body = "\n".join(l for l in src.splitlines()
                     if l.strip() not in ('#include "kargs.hpp"', '#include "jit_kernel.hpp"'))
    gen = tmp_path / f"{name}.inc"
    gen.write_text(body)
    exe = str(tmp_path / name)
    subprocess.run([cxx, "-O1", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(HERE, "cpu_math", "shim"),
                    f'-DAMI_GENERATED="{gen}"', os.path.join(HERE, "cpu_math", "jit_check_complex.cpp"),
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
