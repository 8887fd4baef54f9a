"""The two-pass specialized forward on the CPU: the generated functions of
its two kernels (group sums stored per sample; per frequency, reciprocals
and group products against them) compiled with the host compiler and driven
through the kernels' steps, against the oracle's values -- for solutions too
large for the one-pass kernel, for a small one, on both inputs, and for
poles of higher order."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy, real_freqs, uniform_energies
from oracle.evaluate import energies_from_k

from parity import check, far_from_poles, oracle_terms, reference
from test_multipole_cpu import CASES as MULTIPOLE, _oracle

amd = pytest.importorskip("paper_2311_17189_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


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
                    f'-DAMI_GENERATED="{gen}"', os.path.join(HERE, "cpu_math", "jit_check_two_pass.cpp"),
                    "-o", exe], check=True, capture_output=True, text=True)
    return exe


def _run(exe, beta, t, mu, q, w, inputs):
    w = np.asarray(w).reshape(len(w), -1)
    lines = [f"{len(inputs)} {w.shape[0]} {beta!r} 0.0 {t!r} {mu!r}",
             " ".join(repr(float(v)) for v in np.asarray(q).ravel()[:2 * w.shape[1]]),
             " ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in w.ravel())]
    for row in inputs:
        lines.append(" ".join(repr(float(v)) for v in row))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    out = np.array([[float(v) for v in l.split()] for l in res.stdout.strip().splitlines()])
    return (out[:, 0::2] + 1j * out[:, 1::2]).T


@pytest.mark.parametrize("order,i,n", [(4, 1, 200), (6, 0, 40), (6, 11, 60)])
def test_two_pass_energy_input(order, i, n, tmp_path):
    d = random_self_energy(order, (5, order, i)) if order == 6 else random_self_energy(order, (0, order, i))
    T = amd.Terms.from_diagram(d)
    src = T.source(momentum=False, two_pass=True)
    assert "group_sums_store" in src and "group_accumulate" in src and "void leaf_cotangents(" not in src
    exe = _harness(src, tmp_path, f"tp{order}_{i}")
    beta = 5.0
    E = uniform_energies(n, d.n_eps, seed=(95, order, i), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta), real_freqs(1, 0.4, 0.4, 0.05)])
    terms = oracle_terms(d)
    E = np.ascontiguousarray(E[far_from_poles(terms, d.n_int, E, w)])
    got = _run(exe, beta, 1.0, 0.0, np.zeros(2), w, E)
    ref, scale, dist = reference(d, E, w, beta, terms=terms)
    check(got, ref, scale, dist, label=f"two-pass order {order} energies")


def test_two_pass_momentum_input(tmp_path):
    d = random_self_energy(6, (5, 6, 0))
    T = amd.Terms.from_diagram(d)
    assert T.info()["T"] > 1024
    exe = _harness(T.source(momentum=True, two_pass=True), tmp_path, "tpk")
    beta, t, mu = 5.0, 1.0, 0.1
    q = np.array(DEFAULT_Q)
    w = matsubara_freqs(2, beta)
    terms = oracle_terms(d)
    k = k_samples(50, d.n_int, seed=(96, 6))
    keep = far_from_poles(terms, d.n_int, energies_from_k(d.alpha, k, q, t, mu), w)
    k = np.ascontiguousarray(k[keep])
    got = _run(exe, beta, t, mu, q, w, k)
    E = energies_from_k(d.alpha, k, q, t, mu)
    ref, scale, dist = reference(d, E, w, beta, terms=terms)
    check(got, ref, scale, dist, label="two-pass order 6 momenta")


@pytest.mark.parametrize("name", ["o4", "later"])
def test_two_pass_multipole(name, tmp_path):
    alpha, eps, n_int, ferm = MULTIPOLE[name]
    T = amd.Terms(alpha, eps, n_int, ferm, multipole=True)
    exe = _harness(T.source(momentum=False, two_pass=True), tmp_path, f"tpm_{name}")
    beta = 4.0
    E = uniform_energies(150, eps.shape[1], seed=(97, n_int), a=3.0)
    w = np.concatenate([matsubara_freqs(2, beta) if ferm[-1] else 2j * np.pi * np.arange(1, 3) / beta,
                        real_freqs(1, 0.6, 0.6, 0.05)])
    terms = _oracle(MULTIPOLE[name])
    E = np.ascontiguousarray(E[far_from_poles(terms, n_int, E, w)])
    got = _run(exe, beta, 1.0, 0.0, np.zeros(2), w, E)
    import types
    ref, scale, dist = reference(types.SimpleNamespace(n_int=n_int), E, w, beta, terms=terms)
    check(got, ref, scale, dist, label=f"two-pass multipole {name}")


def test_two_pass_limits_and_chunk_setting():
    big = amd.Terms.from_diagram(random_self_energy(6, (5, 6, 2)))
    assert big.info()["T"] == 2804
    assert "group_sums_store" in big.source(momentum=True, two_pass=True)
    with pytest.raises(amd.AmiError) as e:
        big.source(momentum=True)                    # one-pass: more than 1024 terms
    assert e.value.code == -7
    with pytest.raises(amd.AmiError) as e:
        amd.set_two_pass_chunk_bytes(1000)
    assert e.value.code == -1
    amd.set_two_pass_chunk_bytes(1 << 30)
