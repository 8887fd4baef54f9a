"""Pins of the oracle's symbolic construction (CPU only)."""
import os

import numpy as np
import pytest

from ami_inputs import order2_example, random_self_energy, relabel
from oracle.construct import (CoeffError, LabelError, MultipoleError, canonical,
                              construct, construct_tree, expand_tree, serialize)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_terms(path):
    terms = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        s, leaves, dens = line.split("|")
        lv = []
        for leaf in leaves.split(";"):
            v = [int(x) for x in leaf.split()]
            lv.append((v[0], tuple(v[1:])))
        d = [int(x) for x in dens.split()]
        terms.append((int(s), tuple(lv), ((tuple(d[:3]), tuple(d[3:])),)))
    return terms


def test_order2_term_list_matches_hand_derivation():
    d = order2_example()
    got = canonical(construct(d.alpha, d.eps, d.n_int))
    want = _read_terms(os.path.join(GOLDEN, "order2_terms.txt"))
    assert got == want


def test_order2_tree_is_product_of_two_sums():
    """Fig. 1: the factorized second-order solution is one term whose tree is
    a product node over two sum nodes of two leaves each."""
    d = order2_example()
    tt = construct_tree(d.alpha, d.eps, d.n_int)
    assert len(tt) == 1
    node, dens = tt[0]
    assert node[0] == "*" and len(node[1]) == 2
    for child in node[1]:
        assert child[0] == "+" and len(child[1]) == 2
        assert all(c[1][0] == "leaf" for c in child[1])
        assert sorted(c[0] for c in child[1]) == [-1, 1]
    assert dens == (((1, -1, 1), (0, 0, 1)),)


@pytest.mark.parametrize("order,i", [(3, 0), (3, 2), (4, 1), (4, 3), (5, 0), (5, 5)])
def test_tree_expands_to_flat_list(order, i):
    d = random_self_energy(order, (0, order, i))
    flat = canonical(construct(d.alpha, d.eps, d.n_int))
    tree = construct_tree(d.alpha, d.eps, d.n_int)
    assert canonical(expand_tree(tree)) == flat
    assert len(tree) <= len(flat)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_term_shape_invariants(order):
    """Each sum removes one denominator and adds one leaf; afterwards no
    denominator holds a summed frequency (Sec. 2.2)."""
    for i in range(3):
        d = random_self_energy(order, (1, order, i))
        terms = construct(d.alpha, d.eps, d.n_int)
        for s, leaves, dens in terms:
            assert s in (1, -1)
            assert len(leaves) == order
            assert len(dens) == d.n_g - order
            for e, a in dens:
                assert not any(a[:order])
            for sigma, e in leaves:
                assert sigma in (1, -1)


def test_residue_count_single_sum():
    """One sum over a product of k propagators that all hold nu_1 gives k
    terms (one pole each, Eq. (3))."""
    alpha = np.array([[1, 0], [1, 1], [-1, 1]])
    eps = np.eye(3, dtype=int)
    terms = construct(alpha, eps, 1)
    assert len(terms) == 3
    assert sorted(t[0] for t in terms) == [-1, 1, 1]


def test_bose_leaf_parity_rule():
    """A pole whose frequency part is one fermionic frequency gives a
    Bose-type leaf; an even number gives a Fermi leaf."""
    # G1 = 1/(i nu1 + E1), G2 = 1/(i nu1 + i nu_ext + E2), external fermionic
    alpha = np.array([[1, 0], [1, 1]])
    eps = np.eye(2, dtype=int)
    terms = construct(alpha, eps, 1, fermionic=[1, 1])
    sig = {t[1][0][1]: t[1][0][0] for t in terms}
    assert sig[(-1, 0)] == 1       # pole -E1: no frequency part
    assert sig[(0, -1)] == -1      # pole -E2 - i nu_ext: one fermionic frequency
    # same with a bosonic external frequency: both Fermi
    terms = construct(alpha, eps, 1, fermionic=[1, 0])
    assert all(t[1][0][0] == 1 for t in terms)


def test_serialize_layout():
    d = order2_example()
    terms = canonical(construct(d.alpha, d.eps, d.n_int))
    buf = serialize(terms, 2, 3, 3)
    assert buf[:4] == [2, 3, 3, 4]
    per_term = 1 + 2 * (1 + 3) + 1 * (3 + 3)
    assert len(buf) == 4 + 4 * per_term
    assert buf[4:4 + per_term] == [-1, -1, -1, 0, -1, 1, -1, 0, 0, 1, -1, 1, 0, 0, 1]


def test_errors():
    eps = np.eye(2, dtype=int)
    with pytest.raises(LabelError):
        construct(np.array([[2, 0], [0, 1]]), eps, 1)
    with pytest.raises(LabelError):       # nu_1 in no propagator
        construct(np.array([[0, 1], [0, 1]]), eps, 1)
    with pytest.raises(LabelError):       # summing a bosonic frequency
        construct(np.array([[1, 0], [1, 1]]), eps, 1, fermionic=[0, 1])
    with pytest.raises(MultipoleError):   # identical propagators: double pole
        construct(np.array([[1, 1], [1, 1]]), np.array([[1, 0], [1, 0]]), 1)
    # nu1+nu2 and nu1-nu2: after the first sum nu2 has coefficient 2
    with pytest.raises(CoeffError):
        construct(np.array([[1, 1, 0], [1, -1, 0], [0, 1, 1]]), np.eye(3, dtype=int), 2)


def test_summation_order_changes_terms_not_count_of_leaves():
    """Relabelling the summed frequencies gives another valid term list
    (values are compared in the value tests)."""
    d = random_self_energy(3, (0, 3, 0))
    a = canonical(construct(d.alpha, d.eps, d.n_int))
    r = relabel(d, [2, 0, 1])
    b = canonical(construct(r.alpha, r.eps, r.n_int))
    assert all(len(t[1]) == 3 for t in b)
    assert len(a) > 0 and len(b) > 0
