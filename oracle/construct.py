"""Oracle: symbolic construction of the AMI solution (test infrastructure only).

Follows Sec. 2.2 of Burke & LeBlanc (arXiv 2311.17189):

* the integrand Eq. (1) is a product of propagators Eq. (2),
  ``G_j = 1 / (X_j + eps_j)`` with ``X_j = sum_l alpha_jl * i*nu_l`` and
  ``eps_j = sum_i epsilon_ji * E_i``;
* each Matsubara sum is done with the residue theorem Eq. (3), multiplying the
  residue at every pole Eq. (4) by the Fermi function of that pole;
* the sums are done for ``nu_1 .. nu_n`` in order, the external frequency(s)
  being the last slots (Sec. 5.1.1);
* the result is a list of terms ``A * FT * R`` (Eq. (6)); with factorization
  off the Fermi tree is a plain product of leaves (Sec. 2.2, the FACTORIZE
  paragraph), with it on, terms sharing ``R`` are collected into a tree of
  ``+``/``x``/leaf nodes (Sec. 2.1, Fig. 1).

Readings taken where the paper is silent (each listed in the design notes):

* pole: the zero of ``alpha_p z + (rest of the denominator)``, i.e.
  ``z = -alpha_p * (eps_j + sum_{l != p} alpha_l i nu_l)`` for ``alpha_p = +-1``
  (Eq. (4) read with the sign convention of Eq. (2));
* Fermi or Bose leaf: once the pole's frequency part is fixed,
  ``exp(beta * i nu) = -1`` for a fermionic and ``+1`` for a bosonic frequency,
  so ``f(z) = 1/(sigma exp(beta x) + 1)`` with ``x`` the pole's energy part and
  ``sigma = (-1)^(sum of the pole's fermionic frequency coefficients)``:
  ``sigma = +1`` is the Fermi function, ``sigma = -1`` is ``-n_B``;
* a summation coefficient other than +-1 is rejected; two or more
  denominators with their pole at the same place (a pole of order M, Eq. (5))
  are rejected unless ``multipole=True``, which takes the residue of Eq. (5):
  with ``D_r = c_r (z - z0)`` for the M denominators of the pole,
  ``(z - z0)^M f(beta z) prod_q 1/D_q = prod_r c_r * f(beta z) prod_{other q} 1/D_q``
  and the (M-1)-th derivative by the Leibniz rule gives, for every split
  ``j + sum_q k_q = M - 1``, the term
  ``prod_r c_r * T_j(x0) * prod_q (-a_q)^k_q C(m_q + k_q - 1, k_q) D_q(z0)^-(m_q + k_q)``
  where ``a_q`` is the coefficient of ``nu_p`` in ``D_q``, ``m_q`` its
  multiplicity, and ``T_j(x) = (1/j!) d^j/dx^j f(beta x)`` the j-th Taylor
  coefficient of the pole's Fermi/Bose function at its energy part ``x0``
  (the frequency part again drops out by periodicity).

Data model (plain Python tuples of ints):

* denominator ``(e, a)``: ``e`` energy coefficients (length nE), ``a`` frequency
  coefficients (length nF); its value is ``sum a_l w_l + sum e_i E_i``; a term
  holds its denominators as a multiset (a repeated entry is a power);
* leaf ``(code, e)``: ``code = sigma * (1 + j)``: the Taylor coefficient
  ``T_j`` of ``f_sigma(beta * sum e_i E_i)`` (``j = 0``: the function itself);
* term ``(s, leaves, dens)``: ``s * prod(leaves) / prod(dens)``.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

Den = Tuple[Tuple[int, ...], Tuple[int, ...]]
Leaf = Tuple[int, Tuple[int, ...]]
Term = Tuple[int, Tuple[Leaf, ...], Tuple[Den, ...]]


class AmiError(Exception):
    """Base class of construction errors."""


class LabelError(AmiError):
    """Invalid labels: coefficients outside {-1,0,1}, a summed frequency that
    is bosonic, or a sum over a frequency that no denominator contains."""


class CoeffError(AmiError):
    """A summed frequency appears with a coefficient other than +-1."""


class MultipoleError(AmiError):
    """Two denominators share a pole (pole of order > 1, Eq. (5))."""


def make_r0(alpha, eps) -> Tuple[Den, ...]:
    """The starting integrand R0 as a tuple of denominators (Sec. 5.1.1)."""
    alpha = np.asarray(alpha)
    eps = np.asarray(eps)
    return tuple((tuple(int(x) for x in eps[j]), tuple(int(x) for x in alpha[j]))
                 for j in range(alpha.shape[0]))


def validate(alpha, eps, n_int: int, fermionic=None) -> np.ndarray:
    """Check the labels; returns the fermionic mask as a tuple of 0/1."""
    alpha = np.asarray(alpha)
    eps = np.asarray(eps)
    if alpha.ndim != 2 or eps.ndim != 2 or alpha.shape[0] != eps.shape[0]:
        raise LabelError("alpha and eps must be [nG, nF] and [nG, nE]")
    if alpha.shape[0] < 1:
        raise LabelError("empty integrand")
    n_freq = alpha.shape[1]
    if not (0 <= n_int <= n_freq):
        raise LabelError("n_int out of range")
    if np.any(np.abs(alpha) > 1):
        raise LabelError("alpha coefficients must be -1, 0 or 1")
    if np.any(np.abs(eps) > 1):
        raise LabelError("epsilon coefficients must be -1, 0 or 1")
    if fermionic is None:
        fermionic = np.ones(n_freq, dtype=np.int64)
    fermionic = tuple(int(bool(x)) for x in np.asarray(fermionic).reshape(-1))
    if len(fermionic) != n_freq:
        raise LabelError("fermionic mask has the wrong length")
    if any(fermionic[p] == 0 for p in range(n_int)):
        raise LabelError("only fermionic frequencies can be summed (Eq. (3))")
    return fermionic


def _splits(total: int, n: int):
    """Every tuple of n non-negative integers summing to total."""
    if n == 0:
        if total == 0:
            yield ()
        return
    for k in range(total + 1):
        for rest in _splits(total - k, n - 1):
            yield (k,) + rest


def _binom(n: int, k: int) -> int:
    out = 1
    for i in range(k):
        out = out * (n - i) // (i + 1)
    return out


def sum_one_frequency(term: Term, p: int, fermionic: Sequence[int], multipole: bool = False) -> List[Term]:
    """Apply the residue theorem Eq. (3) to the sum over ``nu_p`` of one term.

    Every denominator with a non-zero coefficient of ``nu_p`` has its pole
    (Eq. (4)); the new term takes the residue factor ``1/c = c``, the
    Fermi/Bose leaf of the pole, and the other denominators evaluated at the
    pole.  The frequency part of the pole is dropped from the leaf
    (``exp(beta i nu)`` is -1 or +1) and kept in the substituted denominators.
    Denominators sharing a pole make it a pole of higher order: rejected, or
    with ``multipole`` taken by Eq. (5) as described in the module notes.
    """
    s, leaves, dens = term
    n_freq = len(dens[0][1]) if dens else 0
    P = [r for r, (_, a) in enumerate(dens) if a[p] != 0]
    if not P:
        raise LabelError(f"no denominator depends on summed frequency {p}")
    poles: Dict[Den, List[int]] = {}
    for r in P:
        e_r, a_r = dens[r]
        c = a_r[p]
        if c not in (1, -1):
            raise CoeffError(f"coefficient {c} of summed frequency {p}")
        e_z = tuple(-c * x for x in e_r)
        a_z = tuple(0 if l == p else -c * a_r[l] for l in range(n_freq))
        if (e_z, a_z) in poles and not multipole:
            raise MultipoleError(f"two denominators share a pole in frequency {p}")
        poles.setdefault((e_z, a_z), []).append(r)
    out: List[Term] = []
    for (e_z, a_z), group in poles.items():
        M = len(group)
        pref = s
        for r in group:
            pref *= dens[r][1][p]
        parity = sum(a_z[l] for l in range(n_freq) if fermionic[l]) % 2
        sigma = 1 if parity == 0 else -1
        # the other denominators at the pole, with their multiplicities and nu_p coefficients
        fixed, moving = [], {}
        for q, (e_q, a_q) in enumerate(dens):
            if q in group:
                continue
            m = a_q[p]
            if m == 0:
                fixed.append((e_q, a_q))
                continue
            e_new = tuple(e_q[i] + m * e_z[i] for i in range(len(e_q)))
            a_new = tuple(0 if l == p else a_q[l] + m * a_z[l] for l in range(n_freq))
            key = ((e_new, a_new), m)
            moving[key] = moving.get(key, 0) + 1
        mkeys = list(moving)
        for split in _splits(M - 1, 1 + len(mkeys)):
            j, ks = split[0], split[1:]
            coef = pref
            new_dens = list(fixed)
            for (den, a), mult, k in zip(mkeys, (moving[x] for x in mkeys), ks):
                coef *= (-a) ** k * _binom(mult + k - 1, k)
                new_dens.extend([den] * (mult + k))
            out.append((coef, leaves + ((sigma * (1 + j), e_z),), tuple(new_dens)))
    return out


def construct(alpha, eps, n_int: int, fermionic=None, multipole: bool = False) -> List[Term]:
    """Flat (FACTORIZE=false) solution: repeated residues over nu_1..nu_n.

    Returns the raw term list, in the order the residues produce it.  With
    ``multipole``, poles of higher order are taken by Eq. (5).
    """
    fermionic = validate(alpha, eps, n_int, fermionic)
    terms: List[Term] = [(1, (), make_r0(alpha, eps))]
    for p in range(n_int):
        nxt: List[Term] = []
        for t in terms:
            nxt.extend(sum_one_frequency(t, p, fermionic, multipole))
        terms = nxt
    for _, _, dens in terms:
        for e, a in dens:
            if not any(e) and not any(a):
                raise MultipoleError("a denominator vanished identically")
    return terms


def _normalize_den(den: Den) -> Tuple[int, Den]:
    """Sign-normalize a denominator: first non-zero of (e..., a...) positive."""
    e, a = den
    for x in e + a:
        if x != 0:
            if x < 0:
                return -1, (tuple(-y for y in e), tuple(-y for y in a))
            return 1, den
    return 1, den


def canonical(terms: Sequence[Term]) -> List[Term]:
    """Canonical form of a flat term list.

    Each denominator is sign-normalized (``1/(-x) = -1/x`` moves the sign into
    the prefactor); leaves are left as they are, since ``f(-y) = 1 - f(y)``
    is not a multiple of ``f(y)``.  Leaves are sorted by ``(sigma, e)``,
    denominators by ``(e, a)``; terms equal in both are merged by adding their
    prefactors, zero prefactors dropped, and the terms sorted by
    ``(leaves, dens)``.
    """
    merged: Dict[Tuple[Tuple[Leaf, ...], Tuple[Den, ...]], int] = {}
    for s, leaves, dens in terms:
        sign = 1
        nd = []
        for d in dens:
            g, d2 = _normalize_den(d)
            sign *= g
            nd.append(d2)
        key = (tuple(sorted(leaves)), tuple(sorted(nd)))
        merged[key] = merged.get(key, 0) + s * sign
    out = [(s, k[0], k[1]) for k, s in merged.items() if s != 0]
    out.sort(key=lambda t: (t[1], t[2]))
    return out


def serialize(terms: Sequence[Term], n_int: int, n_eps: int, n_freq: int) -> List[int]:
    """Flat int32 stream of a canonical term list.

    Header ``n_int, nE, nF, T``; then per term ``s``, ``n_int`` leaves as
    ``code, e[0..nE)``, and the denominators as ``e[0..nE), a[0..nF)``.
    When the terms do not all hold the same number of denominators (poles of
    higher order), the header's ``T`` is written as ``-T`` and every term's
    ``s`` is followed by its number of denominators.
    """
    counts = {len(d) for _, _, d in terms}
    extended = len(counts) > 1
    out = [n_int, n_eps, n_freq, -len(terms) if extended else len(terms)]
    for s, leaves, dens in terms:
        out.append(int(s))
        if extended:
            out.append(len(dens))
        for sigma, e in leaves:
            out.append(int(sigma))
            out.extend(int(x) for x in e)
        for e, a in dens:
            out.extend(int(x) for x in e)
            out.extend(int(x) for x in a)
    return out


# ---------------------------------------------------------------------------
# Factorized Fermi tree (FACTORIZE = true), Sec. 2.1 and Fig. 1
# ---------------------------------------------------------------------------
# A node is one of
#   ("one",)                        the empty product
#   ("leaf", sigma, e)              f_sigma(beta * e.E)
#   ("*", (child, ...))             product of children
#   ("+", ((coef, child), ...))     integer-weighted sum of children
# A tree term is (node, dens); its value is node * prod(1/dens).

ONE = ("one",)


def construct_tree(alpha, eps, n_int: int, fermionic=None):
    """Factorized solution: after each sum, the poles taken from one parent
    term that leave the same remaining denominators (up to sign) are summed
    into one ``+`` node multiplying the parent's tree, and tree terms of
    different parents with the same denominators are joined by a ``+`` node.

    The grouping is this module's reading of Sec. 2.1/2.2 (the paper does not
    fix the tree's shape); only its expansion and its values are pinned.
    """
    fermionic = validate(alpha, eps, n_int, fermionic)
    tterms = [(ONE, make_r0(alpha, eps))]
    for p in range(n_int):
        grouped: Dict[Tuple[Den, ...], list] = {}
        order: List[Tuple[Den, ...]] = []
        for node, dens in tterms:
            children = sum_one_frequency((1, (), dens), p, fermionic)
            local: Dict[Tuple[Den, ...], list] = {}
            local_order = []
            for c, (leaf,), nd in children:
                sign = 1
                norm = []
                for d in nd:
                    g, d2 = _normalize_den(d)
                    sign *= g
                    norm.append(d2)
                key = tuple(sorted(norm))
                if key not in local:
                    local[key] = []
                    local_order.append(key)
                local[key].append((c * sign, ("leaf", leaf[0], leaf[1])))
            for key in local_order:
                factor = ("+", tuple(local[key]))
                new = factor if node == ONE else ("*", (node, factor))
                if key not in grouped:
                    grouped[key] = []
                    order.append(key)
                grouped[key].append(new)
        tterms = []
        for key in order:
            parts = grouped[key]
            node = parts[0] if len(parts) == 1 else ("+", tuple((1, q) for q in parts))
            tterms.append((node, key))
    return tterms


def _expand_node(node):
    """Distribute a tree node into a list of (coef, leaves-tuple)."""
    kind = node[0]
    if kind == "one":
        return [(1, ())]
    if kind == "leaf":
        return [(1, ((node[1], node[2]),))]
    if kind == "*":
        acc = [(1, ())]
        for child in node[1]:
            sub = _expand_node(child)
            acc = [(c1 * c2, l1 + l2) for c1, l1 in acc for c2, l2 in sub]
        return acc
    if kind == "+":
        out = []
        for coef, child in node[1]:
            out.extend((coef * c, l) for c, l in _expand_node(child))
        return out
    raise ValueError(kind)


def expand_tree(tterms) -> List[Term]:
    """Flat terms of a factorized solution (not canonicalized)."""
    out: List[Term] = []
    for node, dens in tterms:
        for c, leaves in _expand_node(node):
            out.append((c, leaves, dens))
    return out


def tree_size(tterms) -> int:
    """Number of nodes in the factorized solution (shared subtrees counted once)."""
    seen = set()

    def visit(node):
        if id(node) in seen:
            return
        seen.add(id(node))
        if node[0] == "*":
            for c in node[1]:
                visit(c)
        elif node[0] == "+":
            for _, c in node[1]:
                visit(c)

    for node, _ in tterms:
        visit(node)
    return len(seen)
