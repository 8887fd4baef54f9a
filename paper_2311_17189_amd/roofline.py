"""Algorithmic FLOP and byte model of one evaluation launch (accounting only).

Counts are those of the evaluation as the library structures it: every
distinct leaf and denominator once per sample (per sample and frequency for
denominators), the Fermi-tree products of each term once per sample (they do
not depend on the external frequency, Sec. 2.3), and one product of
denominator reciprocals per group of terms sharing them.  Only non-zero
integer coefficients are counted.  FMA counts 2 FLOPs; the elementary
functions count the FP64 FLOPs of this build's device-library sequences on
gfx950 (FMA = 2, add/mul/ldexp/rndne/rcp = 1, compares and conversions 0):

    exp 29, expm1 34, IEEE division 17, cos 58 (|x| < 2^30 path)

A term-evaluation is one canonical flat term at one (sample, frequency) point.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C_EXP = 29
C_EXPM1 = 34
C_DIV = 17
C_COS = 58
C_SIN = 58

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


def structure_from_canonical(stream) -> Structure:
    """Distinct leaves, distinct denominators and denominator groups of the
    canonical term stream (layout of ``amiTermsCanonical``)."""
    s = [int(x) for x in np.asarray(stream).reshape(-1)]
    n_int, n_eps, n_freq, T = s[:4]
    per_den = n_eps + n_freq
    per_leaf = 1 + n_eps
    per_term = (len(s) - 4) // T if T else 0
    dpt = (per_term - 1 - n_int * per_leaf) // per_den if T else 0
    pos = 4
    leaves, dens, groups = {}, {}, {}
    for _ in range(T):
        pos += 1
        for _ in range(n_int):
            leaves[(s[pos], tuple(s[pos + 1:pos + per_leaf]))] = True
            pos += per_leaf
        gk = []
        for _ in range(dpt):
            e = tuple(s[pos:pos + n_eps])
            a = tuple(s[pos + n_eps + n_int:pos + per_den])
            dens[(e, a)] = True
            gk.append((e, a))
            pos += per_den
        gk = tuple(sorted(gk))
        groups[gk] = groups.get(gk, 0) + 1
    return Structure(n_int=n_int, n_eps=n_eps, n_freq=n_freq, T=T,
                     leaves=list(leaves), dens=list(dens),
                     groups=[(c, dpt) for c in groups.values()])


def _nnz(v) -> int:
    return sum(1 for x in v if x != 0)


def forward_flops(st: Structure, n_e: int, n_f: int, line_alpha=None) -> dict:
    """FLOPs of one forward launch; ``line_alpha`` (int [nG, nF]) adds the
    energies-from-momenta stage (Sec. 5.2) of the Hubbard path."""
    per_sample = 0
    if line_alpha is not None:
        for row in np.asarray(line_alpha):
            nz = _nnz(row)
            per_sample += 2 * max(nz - 1, 0) + 2 * C_COS + 3
    for sigma, e in st.leaves:
        base = max(_nnz(e) - 1, 0) + 1 + C_DIV
        per_sample += base + (C_EXP + 1 if sigma == 1 else C_EXPM1)
    for n_terms, _ in st.groups:
        per_sample += n_terms * (max(st.n_int - 1, 0) + 1)
    per_point = 0
    for e, a in st.dens:
        per_point += max(_nnz(e) - 1, 0) + 2 * _nnz(a) + 3 + C_DIV + 2
    for n_terms, dpt in st.groups:
        per_point += 6 * max(dpt - 1, 0) + 4
    total = n_e * per_sample + n_e * n_f * per_point
    return {"per_sample": per_sample, "per_point": per_point, "total": float(total),
            "term_evals": float(st.T) * n_e * n_f}


def forward_bytes(n_e: int, n_f: int, n_in_per_sample: int, want_out: bool) -> float:
    """Compulsory HBM bytes of one forward launch: inputs once, outputs once."""
    return float(n_e * n_in_per_sample * 8 + (n_e * n_f * 16 if want_out else 0))
