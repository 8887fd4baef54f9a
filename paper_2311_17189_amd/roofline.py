"""Algorithmic FLOP model of one evaluation launch (accounting only).

Counts are those of the evaluation as the library structures it: every
distinct leaf once per sample, every distinct denominator once per sample and
frequency, the Fermi-tree products of each term once per sample (they do not
depend on the external frequency, Sec. 2.3), one product of denominator
reciprocals per group of terms sharing them, and on the momentum path the
energies from momenta (Sec. 5.2).  Only non-zero integer coefficients count.
FMA counts 2 FLOPs; each elementary function counts the FP64 FLOPs of the
sequence the kernels execute on gfx950, read from the AMD assembly of small
kernels compiled here (FMA 2; add, mul, min/max, ldexp, rndne, rcp 1;
compares and conversions 0):

    sin and cos of one argument (both, reduced)      44
    cos alone (reduced by pi)                        29
    reduction of a momentum component mod 2 pi        8
    e^z and e^z - 1 of one argument (both)           37
    reciprocal (estimate + two Newton steps)          9
    leaf f(y) with its mirror f(-y), Fermi / Bose    47 / 49
    leaf derivative f'(y)                            48
    leaf at a complex argument, Fermi / Bose        112 / 135

Two models: ``forward_flops``/``adjoint_flops`` for the table-driven (packed)
kernels and ``specialized_forward_flops``/``specialized_adjoint_flops`` for the
generated ones, each counting the arithmetic of its own algorithm (the
specialized adjoint sums the cotangents of each distinct denominator before
scattering them, and takes f'(y) = -f(y) f(-y) from the leaf pair).

A term-evaluation is one canonical flat term at one (sample, frequency) point.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C_SINCOS = 44
C_COS = 29
C_RED2PI = 8
C_EXP = 37
C_RCP = 9
C_LEAF_FERMI = 47
C_LEAF_BOSE = 49
C_LEAF_DERIV = 48
C_LEAF_C_FERMI = 112    # leaf at a complex argument (leaf_complex), Fermi / Bose-type
C_LEAF_C_BOSE = 135

PEAK_FP64_VECTOR = 78.6e12     # 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk
PEAK_HBM = 8.0e12              # bytes/s


@dataclass
class Structure:
    n_int: int
    n_eps: int
    n_freq: int
    T: int
    leaves: list      # distinct (sigma, e-tuple)
    dens: list        # distinct (e-tuple, a_ext-tuple)
    groups: list      # per group: (n_terms, n_dens)
    terms: list = None    # per term in stream order: (group index, prefactor, leaf keys)


def structure_from_canonical(stream) -> Structure:
    """Distinct leaves, distinct denominators and denominator groups of the
    canonical term stream (layout of ``amiTermsCanonical``; with T written as
    -T every term's denominator count follows its prefactor).  Leaves keep
    their codes (sigma (1 + j) for Taylor coefficients)."""
    s = [int(x) for x in np.asarray(stream).reshape(-1)]
    n_int, n_eps, n_freq, T = s[:4]
    extended = T < 0
    T = abs(T)
    per_den = n_eps + n_freq
    per_leaf = 1 + n_eps
    dpt = 0
    if T and not extended:
        dpt = ((len(s) - 4) // T - 1 - n_int * per_leaf) // per_den
    pos = 4
    leaves, dens, groups = {}, {}, {}
    gindex, tlist = {}, []
    for _ in range(T):
        pref = s[pos]
        pos += 1
        nd = dpt
        if extended:
            nd = s[pos]
            pos += 1
        lv = []
        for _ in range(n_int):
            key = (s[pos], tuple(s[pos + 1:pos + per_leaf]))
            leaves[key] = True
            lv.append(key)
            pos += per_leaf
        gk = []
        for _ in range(nd):
            e = tuple(s[pos:pos + n_eps])
            a = tuple(s[pos + n_eps + n_int:pos + per_den])
            dens[(e, a)] = True
            gk.append((e, a))
            pos += per_den
        gk = tuple(sorted(gk))
        groups[gk] = groups.get(gk, 0) + 1
        tlist.append((gindex.setdefault(gk, len(gindex)), pref, tuple(lv)))
    return Structure(n_int=n_int, n_eps=n_eps, n_freq=n_freq, T=T,
                     leaves=list(leaves), dens=list(dens),
                     groups=[(c, len(gk)) for gk, c in groups.items()], terms=tlist)


def _nnz(v) -> int:
    return sum(1 for x in v if x != 0)


def _use_products(st: Structure) -> bool:
    """The kernels build Fermi leaves from products of exp(beta E_i) when the
    Fermi leaves outnumber the energies they use (same rule as the host)."""
    used = set()
    n_fermi = 0
    for sigma, e in st.leaves:
        if sigma == 1:
            n_fermi += 1
            used.update(i for i, x in enumerate(e) if x != 0)
    return n_fermi > len(used)


def _leaf_flops(st: Structure) -> int:
    prod = _use_products(st)
    total = 0
    used = set()
    for sigma, e in st.leaves:
        nz = _nnz(e)
        if sigma == -1:
            total += max(nz - 1, 0) + 2 + C_LEAF_BOSE
        elif prod:
            total += max(nz - 2, 0) + 1 + C_RCP + 1        # N*P products, N+P, 1/(N+P), N*r
            used.update(i for i, x in enumerate(e) if x != 0)
        else:
            total += max(nz - 1, 0) + 1 + C_LEAF_FERMI
    if prod:
        total += len(used) * (1 + C_EXP)                     # exp(beta E_i)
    return total


def _momentum_flops(line_alpha, n_int: int, sincos: bool) -> int:
    """Momenta reduced mod 2 pi, K_j per component, then E_j = 2t(cos K_jx +
    cos K_jy) + mu (cos alone in the forward, sin and cos in the adjoint, which
    also keeps cos K_jx + cos K_jy)."""
    total = 2 * n_int * C_RED2PI
    for row in np.asarray(line_alpha):
        total += 2 * max(_nnz(row) - 1, 0) + 3
        total += 2 * C_SINCOS + 1 if sincos else 2 * C_COS
    return total


def _momentum_flops_added(line_alpha, n_int: int) -> int:
    """The specialized adjoint's energies from momenta: the loop momenta
    reduced mod 2 pi, sin and cos of each loop component, then sin and cos of
    every line component by angle addition (each further term: two products
    and two FMAs, 6 FLOPs; sin and cos of q come from the host), and
    E_j = 2t(cos K_jx + cos K_jy) + mu."""
    total = 2 * n_int * (C_RED2PI + C_SINCOS)
    for row in np.asarray(line_alpha):
        total += 2 * 6 * max(_nnz(row) - 1, 0) + 3
    return total


def _den_flops(st: Structure) -> int:
    total = 0
    for e, a in st.dens:
        total += max(_nnz(e) - 1, 0) + 2 * _nnz(a) + 3 + C_RCP + 2
    return total


def forward_flops(st: Structure, n_e: int, n_f: int, line_alpha=None) -> dict:
    """FLOPs of one forward launch; ``line_alpha`` (int [nG, nF]) adds the
    energies-from-momenta stage (Sec. 5.2) of the momentum path."""
    per_sample = _leaf_flops(st)
    if line_alpha is not None:
        per_sample += _momentum_flops(line_alpha, st.n_int, sincos=False)
    for n_terms, _ in st.groups:
        per_sample += n_terms * (st.n_int + 1)              # n-1 products, sign, accumulate
    per_point = _den_flops(st)
    for n_terms, dpt in st.groups:
        per_point += 6 * max(dpt - 1, 0) + 4
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


def adjoint_flops(st: Structure, n_e: int, n_f: int, line_alpha=None, with_values=False) -> dict:
    """FLOPs of one adjoint launch: the forward recomputation of leaves,
    group sums and reciprocals, then per group and frequency the product of
    its reciprocals, the group-sum cotangent and one complex product per
    denominator scattered to energies and frequencies; per term the
    prefix/suffix products of its leaves; per leaf its derivative scattered
    to energies and beta; on the momentum path the chain rule through
    -2t sin K."""
    ni = st.n_int
    per_sample = _leaf_flops(st)
    if line_alpha is not None:
        per_sample += _momentum_flops(line_alpha, ni, sincos=True)
        for row in np.asarray(line_alpha)[:, :ni]:
            per_sample += 10 + 2 * _nnz(row)
    for n_terms, _ in st.groups:
        per_sample += n_terms * (st.n_int + 1)              # group sums
        per_sample += n_terms * (1 + ni + (ni - 1) + 2 * ni)   # leaf cotangents
    for sigma, e in st.leaves:
        per_sample += max(_nnz(e) - 1, 0) + 2 + C_LEAF_DERIV + 1 + _nnz(e) + 1 + 2
    per_point = _den_flops(st)
    for n_terms, dpt in st.groups:
        per_point += 6 * max(dpt - 1, 0) + 3 + 2 + 6
        per_point += dpt * (6 + 3 + 2)          # rho * u, scatter (about 3 energies, 1 frequency)
        if with_values:
            per_point += 4                      # FT_g R_g accumulated into the value
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


# ---- the specialized (generated) kernels ------------------------------------

def _taylor_flops(j: int) -> int:
    """A Taylor-coefficient leaf of order j from f and f(-y): j monomials of
    degree j + 1 (j products and one FMA each), then beta^j / j!."""
    return j * (j + 2) + j + 1 if j > 0 else 0


def _spec_leaves(st: Structure, adjoint: bool) -> int:
    total = 0
    for code, e in st.leaves:
        sigma = 1 if code > 0 else -1
        total += max(_nnz(e) - 1, 0) + 1 + (1 if sigma == -1 else 0)    # x, beta x, + e_reg
        total += C_LEAF_BOSE if sigma == -1 else C_LEAF_FERMI
        total += _taylor_flops(abs(code) - 1)
        if adjoint:
            total += 1                                                   # f'(y) = -f(y) f(-y)
    return total


def _spec_group_sums(st: Structure) -> int:
    """Group sums as generated: each term's leaves multiplied left to right,
    the last factor of every term but a group's first fused into the
    accumulation (FMA; a unit prefactor's sign is a free negation).  Equal
    leading products of the terms of one group are computed once (the
    compiler merges the identical expressions), so a product counts once per
    distinct prefix."""
    n = st.n_int
    if st.terms is None:
        return sum(n_terms * n - 1 for n_terms, _ in st.groups)
    total, prefixes, seen = 0, set(), set()
    for g, pref, lv in st.terms:
        first = g not in seen
        seen.add(g)
        unit = abs(pref) == 1
        upto = n if (first or not unit) else n - 1       # factors multiplied before the accumulation
        for k in range(2, upto + 1):
            prefixes.add((g, lv[:k]))
        if not first:
            total += 2                                     # fma into the group sum
        if not unit:
            total += 0 if first else 0                     # the prefactor enters the FMA
    return total + len(prefixes)


def _spec_leaf_cotangents(st: Structure) -> int:
    """Leaf cotangents as generated: per term the products FTB_g f_1 ... f_j
    (shared by the terms of a group with the same leading leaves, a unit sign
    being applied in the update), the suffix products (n - 2 multiplies), one
    update per leaf (n - 1 FMAs and an add)."""
    n = st.n_int
    if st.terms is None or n == 0:
        return sum(n_terms * (4 * n - 4) for n_terms, _ in st.groups)
    prefixes, total = set(), 0
    for g, pref, lv in st.terms:
        unit = abs(pref) == 1
        if not unit:
            total += 1 + (n - 1)                           # FTB s, its own prefix chain
        else:
            for k in range(1, n):
                prefixes.add((g, lv[:k]))
        total += max(n - 2, 0) + 2 * (n - 1) + 1
    return total + len(prefixes)


def _spec_dens(st: Structure) -> int:
    total = 0
    for e, a in st.dens:
        na = _nnz(a)
        total += max(_nnz(e) - 1, 0) + na + max(na - 1, 0)   # real and imaginary parts
        total += 3 + C_RCP + 2                                # |D|^2, 1/|D|^2, D* / |D|^2
    for n_terms, dpt in st.groups:
        total += 6 * max(dpt - 1, 0)                          # complex product of the reciprocals
    return total


def specialized_forward_flops(st: Structure, n_e: int, n_f: int, line_alpha=None) -> dict:
    """FLOPs of one forward launch of the generated kernel."""
    per_sample = _spec_leaves(st, False) + _spec_group_sums(st)
    if line_alpha is not None:
        per_sample += _momentum_flops(line_alpha, st.n_int, sincos=False)
    per_point = _spec_dens(st) + 4 * len(st.groups)           # FT_g R_g accumulated
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


def specialized_complex_forward_flops(st: Structure, n_e: int, n_f: int) -> dict:
    """FLOPs of one launch of the complex-energy forward kernel: per sample the
    leaf arguments of the real and imaginary parts, the complex leaf, the
    complex group sums (6 FLOPs per complex product, 2 per accumulation) and
    the imaginary energy part of every denominator; per (sample, frequency)
    the denominators as in the real kernel plus that part, and every group's
    complex FT_g R_g accumulation (8)."""
    n = st.n_int
    per_sample = 0
    for code, e in st.leaves:
        sigma = 1 if code > 0 else -1
        per_sample += 2 * max(_nnz(e) - 1, 0) + 2 + (1 if sigma == -1 else 0)
        per_sample += C_LEAF_C_BOSE if sigma == -1 else C_LEAF_C_FERMI
    per_sample += sum(n_terms * (6 * max(n - 1, 0) + 2) for n_terms, _ in st.groups)
    for e, a in st.dens:
        na = _nnz(a)
        per_sample += max(_nnz(e) + na - 1, 0) + max(na - 1, 0)      # den_args at Im E (w = 0)
    per_point = _spec_dens(st) + len(st.dens) + 8 * len(st.groups)
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


def specialized_adjoint_flops(st: Structure, n_e: int, n_f: int, line_alpha=None,
                              with_values=False) -> dict:
    """FLOPs of one adjoint launch of the generated kernel: the forward
    recomputation, per group and frequency the group-sum cotangent and u_g,
    per distinct denominator the sum of its u_g, one complex product and the
    scatter to energies and frequencies; per term the prefix/suffix products
    of its leaves; per leaf its derivative, the scatter to energies and beta;
    on the momentum path sin and cos of the lines by angle addition and the
    chain rule through -2t sin K."""
    n = st.n_int
    per_sample = _spec_leaves(st, True) + _spec_group_sums(st)
    per_sample += _spec_leaf_cotangents(st)
    for sigma, e in st.leaves:
        per_sample += max(_nnz(e) - 1, 0) + (1 if sigma == -1 else 0)    # x recomputed
        per_sample += 4 + _nnz(e)                                         # f' FB, beta, d/dbeta, scatter
    if line_alpha is not None:
        per_sample += _momentum_flops_added(line_alpha, n)
        for row in np.asarray(line_alpha)[:, :n]:
            per_sample += 8 + 2 * _nnz(row)                               # mu, t, -2t sin K, d/dk
    per_point = _spec_dens(st)
    per_point += len(st.groups) * (4 + 8 + (4 if with_values else 0))
    # each group holds dpt denominator occurrences; U_k sums them per distinct denominator
    n_occ = sum(dpt for _, dpt in st.groups)
    per_point += 2 * max(n_occ - len(st.dens), 0)
    for e, a in st.dens:
        per_point += 6 + _nnz(e) + 2 * _nnz(a)
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


def mc_flops(st: Structure, n_samples: int, n_f: int, line_alpha) -> dict:
    """FLOPs of one Monte-Carlo launch: per sample the word-to-momentum
    mapping (four per component), the specialized forward without its output,
    and per (sample, frequency) four accumulations (two adds, two FMAs)."""
    comps = 2 * st.n_int
    fw = specialized_forward_flops(st, 1, 1, line_alpha)
    per_sample = fw["per_sample"] - 2 * st.n_int * C_RED2PI + 4 * comps
    per_point = fw["per_point"] + 6
    total = float(n_samples) * (per_sample + n_f * per_point)
    return {"per_sample": per_sample, "per_point": per_point, "total": total,
            "term_evals": float(st.T) * n_samples * n_f}
