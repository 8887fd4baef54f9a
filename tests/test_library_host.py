"""Host side of libamigpu (CPU only): the library loads, exports every symbol
of include/amigpu.h, and its C++ construction reproduces the oracle's
canonical term list bit for bit (FACTORIZE off and on)."""
import ctypes
import os
import re

import numpy as np
import pytest

from ami_inputs import order2_example, random_self_energy
from oracle.construct import AmiError as OracleError
from oracle.construct import (CoeffError, LabelError, MultipoleError, canonical,
                              construct, serialize)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amigpu.h")

amd = pytest.importorskip("paper_2311_17189_amd")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ami[A-Z]\w*)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(amd.lib_path())
    syms = _declared_symbols()
    assert len(syms) >= 8
    for name in syms:
        assert hasattr(lib, name), name
    assert "gfx950" in amd.version()


def _oracle_stream(d):
    terms = canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))
    return serialize(terms, d.n_int, d.n_eps, d.n_freq)


def test_order2_bit_exact():
    d = order2_example()
    t = amd.Terms.from_diagram(d, factorize=True)
    want = _oracle_stream(d)
    assert list(t.canonical()) == want
    assert list(t.canonical(from_tree=True)) == want
    info = t.info()
    assert (info["T"], info["L"], info["D"], info["G"]) == (4, 4, 1, 1)
    assert info["tree_nodes"] > 0


@pytest.mark.parametrize("order,count", [(2, 20), (3, 40), (4, 40), (5, 20), (6, 4)])
def test_seeded_diagrams_bit_exact(order, count):
    for i in range(count):
        d = random_self_energy(order, (21, order, i))
        try:
            want = _oracle_stream(d)
        except OracleError as e:
            with pytest.raises(amd.AmiError):
                amd.Terms.from_diagram(d)
            continue
        t = amd.Terms.from_diagram(d, factorize=(i % 2 == 0))
        got = t.canonical()
        assert got.dtype == np.int32
        assert list(got) == want, (order, i)
        if i % 2 == 0:
            assert list(t.canonical(from_tree=True)) == want
        info = t.info()
        assert info["T"] == want[3]
        assert info["leaves_per_term"] == order
        assert info["dens_per_term"] == d.n_g - order


def test_bosonic_external_and_zero_sums():
    alpha = np.array([[1, 0], [1, 1], [-1, 1]])
    eps = np.eye(3, dtype=int)
    for ferm in ([1, 0], [1, 1]):
        t = amd.Terms(alpha, eps, 1, fermionic=ferm)
        want = serialize(canonical(construct(alpha, eps, 1, ferm)), 1, 3, 2)
        assert list(t.canonical()) == want
    # no sums at all: the single term is R0 itself
    t0 = amd.Terms(alpha, eps, 0)
    want = serialize(canonical(construct(alpha, eps, 0)), 0, 3, 2)
    assert list(t0.canonical()) == want


@pytest.mark.parametrize("alpha,eps,n_int,ferm,oracle_exc,status", [
    ([[2, 0], [0, 1]], np.eye(2), 1, None, LabelError, "AMI_E_LABEL"),
    ([[0, 1], [0, 1]], np.eye(2), 1, None, LabelError, "AMI_E_LABEL"),
    ([[1, 0], [1, 1]], np.eye(2), 1, [0, 1], LabelError, "AMI_E_LABEL"),
    ([[1, 1], [1, 1]], [[1, 0], [1, 0]], 1, None, MultipoleError, "AMI_E_MULTIPOLE"),
    ([[1, 1, 0], [1, -1, 0], [0, 1, 1]], np.eye(3), 2, None, CoeffError, "AMI_E_COEFF"),
])
def test_errors_match_oracle(alpha, eps, n_int, ferm, oracle_exc, status):
    alpha = np.array(alpha)
    eps = np.array(eps, dtype=int)
    with pytest.raises(oracle_exc):
        construct(alpha, eps, n_int, ferm)
    with pytest.raises(amd.AmiError) as ei:
        amd.Terms(alpha, eps, n_int, fermionic=ferm)
    assert ei.value.status == status


def test_argument_errors():
    with pytest.raises(amd.AmiError) as ei:
        amd.Terms(np.zeros((0, 2)), np.zeros((0, 2)), 1)
    assert ei.value.status == "AMI_E_ARG"
    with pytest.raises(amd.AmiError) as ei:
        amd.Terms(np.eye(2), np.eye(2), 3)
    assert ei.value.status == "AMI_E_ARG"
