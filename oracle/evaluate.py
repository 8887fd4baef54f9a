"""Oracle: numeric evaluation of the AMI solution (test infrastructure only).

* :func:`evaluate_terms` -- the batched evaluation of Sec. 2.3: a flat term
  list (Eq. (6) with factorization off) over ``N_E`` energy rows and ``N_F``
  external frequency rows, giving the ``[N_F, N_E]`` result of Sec. 2.3.
* :func:`evaluate_tree`  -- the same from the factorized Fermi tree (Sec. 2.1).
* :func:`energies_from_k` -- the momentum mapping of Sec. 5.2 (Kronecker form
  ``A = alpha (x) I_d``, ``K = k A^T``, one dispersion per block of ``d``
  columns) with the 2D Hubbard dispersion ``eps(k) = -2t(cos kx + cos ky) - mu``;
  energies are ``E = -eps`` (Sec. 2.2, below Eq. (2)).
* :func:`gradients` -- analytic derivatives of a cotangent-weighted sum of the
  result with respect to energies (real or complex), beta, external
  frequencies, and through
  :func:`energies_from_k` with respect to momenta and ``mu``.

Arithmetic is numpy ``longdouble`` (x87 80-bit on x86-64) unless a dtype is
passed; nothing is blocked, fused or reordered beyond a loop over terms
vectorized over samples.

Readings: a leaf ``(sigma, e)`` is ``f_sigma(y) = 1/(sigma*exp(y) + 1)`` at
``y = beta*(e . E)``; the regulator ``e_reg`` is added to ``e . E`` of
``sigma = -1`` (Bose-type) leaves only.  Energies may be complex (Sec. 5.1.3: the
energy vector's element type is complex): the leaves and denominators are
then the analytic continuations of the same expressions.  A leaf code ``sigma (1 + j)`` with
``j > 0`` (from a pole of higher order) is the j-th Taylor coefficient of that
function in ``x = e . E`` (:func:`leaf_coefficient`).  A denominator ``(e, a)`` is
``e . E + a_ext . w`` -- internal frequency slots are zero after construction
and are ignored.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

LD = np.longdouble
CLD = np.clongdouble


def leaf_value(sigma: int, y):
    """``f_sigma(y) = 1/(sigma e^y + 1)``; the Bose-type form is written
    ``-1/expm1(y)`` so it keeps full relative precision near ``y = 0``.

    Complex ``y`` (complex energies): with ``u = e^{-y}`` where ``Re y > 0``
    the same function is ``u/(1 + u)`` (Fermi) and ``u/expm1(-y)`` (Bose-type),
    which cannot overflow; elsewhere the forms above are used as they are."""
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        if not np.iscomplexobj(y):
            if sigma == 1:
                return 1 / (np.exp(y) + 1)
            return -1 / np.expm1(y)
        pos = np.real(y) > 0
        z = np.where(pos, -y, y)          # Re z <= 0: e^z cannot overflow
        if sigma == 1:
            u = np.exp(z)
            return np.where(pos, u / (1 + u), 1 / (u + 1))
        m = np.expm1(z)
        return np.where(pos, np.exp(z) / m, -1 / m)


def _derivative_monomials(j: int):
    """f^(j) of a leaf as a polynomial in f and fm = f(-y) = 1 - f:
    {(a, b): c} for c f^a fm^b, from f' = -f fm and fm' = f fm (both kinds)."""
    poly = {(1, 0): 1}
    for _ in range(j):
        nxt = {}
        for (a, b), c in poly.items():
            if a:
                nxt[(a, b + 1)] = nxt.get((a, b + 1), 0) - a * c
            if b:
                nxt[(a + 1, b)] = nxt.get((a + 1, b), 0) + b * c
        poly = {k: v for k, v in nxt.items() if v}
    return poly


def leaf_coefficient(code: int, x, beta):
    """Leaf ``(code, e)`` at ``x = e.E`` (with the regulator already added):
    for ``code = sigma (1 + j)`` the Taylor coefficient
    ``T_j(x) = (1/j!) d^j/dx^j f_sigma(beta x) = beta^j f_sigma^(j)(beta x) / j!``,
    with ``f^(j)`` written through ``f`` and ``f(-y) = 1 - f`` (no cancellation
    where f saturates)."""
    sigma = 1 if code > 0 else -1
    j = abs(code) - 1
    y = beta * x
    f = leaf_value(sigma, y)
    if j == 0:
        return f
    fm = leaf_value(sigma, -y)
    acc = 0
    for (a, b), c in _derivative_monomials(j).items():
        acc = acc + c * f ** a * fm ** b
    fact = 1
    for i in range(2, j + 1):
        fact *= i
    return acc * beta ** j / fact


def _ext_slots(n_int: int, a: Sequence[int]):
    return [int(x) for x in a[n_int:]]


def evaluate_terms(terms, n_int: int, energies, ext_freqs, beta, e_reg=0.0,
                   dtype=LD):
    """Sum of flat terms at every (frequency row, energy row).

    ``energies`` real or complex [N_E, nE]; ``ext_freqs`` complex [N_F, n_ext]
    (or [N_F] for one external slot).  Returns complex [N_F, N_E].  Complex
    energies enter the leaves and the denominators alike: every expression
    is the same analytic function of them.
    """
    cdt = CLD if dtype is LD else np.complex128
    E = np.asarray(energies)
    E = E.astype(cdt if np.iscomplexobj(E) else dtype)
    w = np.asarray(ext_freqs)
    if w.ndim == 1:
        w = w[:, None]
    w = w.astype(cdt)
    beta = dtype(beta)
    e_reg = dtype(e_reg)
    n_e = E.shape[0]
    n_f = w.shape[0]
    out = np.zeros((n_f, n_e), dtype=cdt)
    for s, leaves, dens in terms:
        ft = np.full(n_e, dtype(s), dtype=E.dtype)
        for code, e in leaves:
            x = E @ np.asarray(e, dtype=dtype)
            if code < 0:
                x = x + e_reg
            ft = ft * leaf_coefficient(code, x, beta)
        for f in range(n_f):
            r = np.ones(n_e, dtype=cdt)
            for e, a in dens:
                assert not any(a[:n_int]), "internal slot left after construction"
                d = (E @ np.asarray(e, dtype=dtype)).astype(cdt)
                for j, aj in enumerate(_ext_slots(n_int, a)):
                    if aj:
                        d = d + aj * w[f, j]
                r = r / d
            out[f] += ft * r
    return out


def term_magnitudes(terms, n_int: int, energies, ext_freqs, beta, e_reg=0.0):
    """``sum_t |v_t|`` at every point: the natural scale of the rounding error
    of the sum over terms, used as the denominator of relative errors."""
    E = np.asarray(energies)
    E = E.astype(CLD if np.iscomplexobj(E) else LD)
    w = np.asarray(ext_freqs)
    if w.ndim == 1:
        w = w[:, None]
    w = w.astype(CLD)
    out = np.zeros((w.shape[0], E.shape[0]), dtype=LD)
    for t in terms:
        v = evaluate_terms([t], n_int, E, w, beta, e_reg)
        out += np.abs(v)
    return out


def _eval_node(node, E, beta, e_reg, dtype):
    kind = node[0]
    if kind == "one":
        return np.ones(E.shape[0], dtype=dtype)
    if kind == "leaf":
        x = E @ np.asarray(node[2], dtype=dtype)
        if node[1] == -1:
            x = x + e_reg
        return leaf_value(node[1], beta * x)
    if kind == "*":
        acc = np.ones(E.shape[0], dtype=dtype)
        for child in node[1]:
            acc = acc * _eval_node(child, E, beta, e_reg, dtype)
        return acc
    if kind == "+":
        acc = np.zeros(E.shape[0], dtype=dtype)
        for coef, child in node[1]:
            acc = acc + coef * _eval_node(child, E, beta, e_reg, dtype)
        return acc
    raise ValueError(kind)


def evaluate_tree(tterms, n_int: int, energies, ext_freqs, beta, e_reg=0.0,
                  dtype=LD):
    """Evaluate the factorized solution: each tree once per energy row (it
    does not depend on the external frequencies, Sec. 2.3), times the product
    of its denominators per frequency row."""
    cdt = CLD if dtype is LD else np.complex128
    E = np.asarray(energies).astype(dtype)
    w = np.asarray(ext_freqs)
    if w.ndim == 1:
        w = w[:, None]
    w = w.astype(cdt)
    beta = dtype(beta)
    e_reg = dtype(e_reg)
    out = np.zeros((w.shape[0], E.shape[0]), dtype=cdt)
    for node, dens in tterms:
        ft = _eval_node(node, E, beta, e_reg, dtype)
        for f in range(w.shape[0]):
            r = np.ones(E.shape[0], dtype=cdt)
            for e, a in dens:
                d = (E @ np.asarray(e, dtype=dtype)).astype(cdt)
                for j, aj in enumerate(_ext_slots(n_int, a)):
                    if aj:
                        d = d + aj * w[f, j]
                r = r / d
            out[f] += ft * r
    return out


# ---------------------------------------------------------------------------
# Energies from momenta (Sec. 5.2)
# ---------------------------------------------------------------------------

def kron_alpha(alpha, dim: int = 2) -> np.ndarray:
    """``A = alpha (x) I_d`` (Sec. 5.2)."""
    return np.kron(np.asarray(alpha, dtype=np.int64), np.eye(dim, dtype=np.int64))


def line_momenta(alpha, k_int, q, dim: int = 2, dtype=LD) -> np.ndarray:
    """``K = k A^T`` with ``k = [k_int, 1 q]`` (Sec. 5.2): [N_E, d*nG]."""
    k_int = np.asarray(k_int).astype(dtype)
    n_e = k_int.shape[0]
    q = np.asarray(q).astype(dtype).reshape(1, -1)
    alpha = np.asarray(alpha)
    n_ext = alpha.shape[1] - k_int.shape[1] // dim
    k = np.concatenate([k_int] + [np.repeat(q, n_e, axis=0)] * n_ext, axis=1)
    A = kron_alpha(alpha, dim).astype(dtype)
    return k @ A.T


def hubbard_energy(Kblock, t, mu):
    """``E = -eps(K) = 2t(cos Kx + cos Ky) + mu`` for one [N_E, d] block."""
    return 2 * t * np.cos(Kblock).sum(axis=1) + mu


def energies_from_k(alpha, k_int, q, t=1.0, mu=0.0, dim: int = 2, dtype=LD):
    """Energies of every propagator, [N_E, nG]: one dispersion per block of
    ``d`` columns of ``K`` (Sec. 5.2, last display)."""
    K = line_momenta(alpha, k_int, q, dim, dtype)
    ng = np.asarray(alpha).shape[0]
    t = dtype(t)
    mu = dtype(mu)
    return np.stack([hubbard_energy(K[:, i * dim:(i + 1) * dim], t, mu)
                     for i in range(ng)], axis=1)


# ---------------------------------------------------------------------------
# Gradients
# ---------------------------------------------------------------------------

def gradients(terms, n_int: int, energies, ext_freqs, beta, cot, e_reg=0.0,
              per_sample=False):
    """Derivatives of ``L = Re sum_{f,s} conj(cot[f,s]) * I[f,s]``.

    For one term ``v = s prod_l f_l prod_r 1/D_r`` with ``y_l = beta x_l``:
    ``d ln f_sigma / dy = -(1 - f_sigma(y)) = -f_sigma(-y)``, ``d ln(1/D) / dD = -1/D``, so

    * ``dv/dE_i  = v * [ -beta sum_l e_li (1 - f_l) - sum_r e_ri / D_r ]``
    * ``dv/dbeta = v * [ -sum_l x_l (1 - f_l) ]`` at fixed frequency values
    * ``dv/dw_j  = v * [ -sum_r a_rj / D_r ]`` (holomorphic in ``w``).

    Returns ``(dE [N_E, nE] real, dbeta real, dw [N_F, n_ext] complex)``, the
    complex one in the convention ``conj(dI/dw) * cot`` summed over samples;
    with ``per_sample`` the last two are not summed: ``dbeta [N_E]``,
    ``dw [N_F, N_E, n_ext]``.

    Complex energies (Sec. 5.1.3): every expression above is the same analytic
    function of ``E`` (the leaf's ``d ln f/dy = -f(-y)`` holds at complex
    ``y``), so ``dI/dE`` is complex and ``dE`` is returned complex in the
    convention of ``dw``: ``sum_f cot * conj(dI/dE)``, which is
    ``dL/dRe E + i dL/dIm E`` of the real ``L`` (its real part is the formula
    for real energies).  ``dbeta`` stays real (beta is).
    """
    cplx = np.iscomplexobj(energies)
    E = np.asarray(energies).astype(CLD if cplx else LD)
    w = np.asarray(ext_freqs)
    if w.ndim == 1:
        w = w[:, None]
    w = w.astype(CLD)
    g = np.asarray(cot).astype(CLD)
    beta = LD(beta)
    e_reg = LD(e_reg)
    n_e, n_eps = E.shape
    n_f, n_ext = w.shape
    dE = np.zeros((n_e, n_eps), dtype=E.dtype)
    dbeta = np.zeros(n_e, dtype=LD)
    dw = np.zeros((n_f, n_e, n_ext), dtype=CLD)
    for s, leaves, dens in terms:
        if any(abs(code) > 1 for code, _ in leaves):
            assert not cplx, "Taylor-coefficient leaves are taken at real energies"
            ft, dft_dE, dft_db = _taylor_term_leaves(s, leaves, E, beta, e_reg)
        else:
            ft = np.full(n_e, LD(s), dtype=E.dtype)
            dlnft_dE = np.zeros((n_e, n_eps), dtype=E.dtype)
            dlnft_db = np.zeros(n_e, dtype=E.dtype)
            for sigma, e in leaves:
                ev = np.asarray(e, dtype=LD)
                x = E @ ev
                if sigma == -1:
                    x = x + e_reg
                f = leaf_value(sigma, beta * x)
                ft = ft * f
                # 1 - f_sigma(y) = f_sigma(-y) for both statistics; written this way
                # it keeps full relative precision where f saturates at 1
                one_minus = leaf_value(sigma, -beta * x)
                dlnft_dE -= beta * one_minus[:, None] * ev[None, :]
                dlnft_db -= x * one_minus
            dft_dE = ft[:, None] * dlnft_dE
            dft_db = ft * dlnft_db
        for fi in range(n_f):
            r = np.ones(n_e, dtype=CLD)
            dlnr_dE = np.zeros((n_e, n_eps), dtype=CLD)
            dlnr_dw = np.zeros((n_e, n_ext), dtype=CLD)
            for e, a in dens:
                ev = np.asarray(e, dtype=LD)
                d = (E @ ev).astype(CLD)
                ext = _ext_slots(n_int, a)
                for j, aj in enumerate(ext):
                    if aj:
                        d = d + aj * w[fi, j]
                r = r / d
                dlnr_dE -= ev[None, :] / d[:, None]
                for j, aj in enumerate(ext):
                    if aj:
                        dlnr_dw[:, j] -= aj / d
            v = ft * r
            gf = g[fi]
            dv_dE = dft_dE * r[:, None] + v[:, None] * dlnr_dE
            if cplx:
                dE += gf[:, None] * np.conj(dv_dE)
            else:
                dE += np.real(np.conj(gf)[:, None] * dv_dE)
            dbeta += np.real(np.conj(gf) * r * dft_db)
            dv_dw = v[:, None] * dlnr_dw
            dw[fi] += gf[:, None] * np.conj(dv_dw)
    if per_sample:
        return dE, dbeta, dw
    return dE, np.sum(dbeta), np.sum(dw, axis=1)


def _taylor_term_leaves(s, leaves, E, beta, e_reg):
    """The Fermi-tree product ``s prod_l T_l`` of a term holding
    Taylor-coefficient leaves (poles of higher order, Eq. (5)) and its
    derivatives by the product rule, since a ``T_j`` can vanish.  With
    ``T_j(x) = beta^j f^(j)(beta x) / j!`` (``leaf_coefficient``):
    ``dT_j/dx = (j + 1) T_(j+1)`` and ``dT_j/dbeta = (j T_j + x (j + 1) T_(j+1)) / beta``
    (the code of ``T_(j+1)`` is ``sigma (j + 2)``); x holds the regulator of a
    Bose-type leaf.  Returns ``(ft [N_E], dft/dE [N_E, nE], dft/dbeta [N_E])``."""
    n_e, n_eps = E.shape
    vals, dx, db, evs = [], [], [], []
    for code, e in leaves:
        sigma = 1 if code > 0 else -1
        j = abs(code) - 1
        ev = np.asarray(e, dtype=LD)
        x = E @ ev
        if sigma == -1:
            x = x + e_reg
        t = leaf_coefficient(code, x, beta)
        slope = (j + 1) * leaf_coefficient(sigma * (j + 2), x, beta)
        vals.append(t)
        dx.append(slope)
        db.append((j * t + x * slope) / beta)
        evs.append(ev)
    ft = np.full(n_e, LD(s), dtype=LD)
    for t in vals:
        ft = ft * t
    dft_dE = np.zeros((n_e, n_eps), dtype=LD)
    dft_db = np.zeros(n_e, dtype=LD)
    for i in range(len(vals)):
        rest = np.full(n_e, LD(s), dtype=LD)
        for m, t in enumerate(vals):
            if m != i:
                rest = rest * t
        dft_dE += (rest * dx[i])[:, None] * evs[i][None, :]
        dft_db += rest * db[i]
    return ft, dft_dE, dft_db


def momentum_gradients(alpha, k_int, q, t, mu, dE, dim: int = 2):
    """Chain rule through :func:`energies_from_k`:
    ``dE_j/dK_jc = -2t sin K_jc``, ``K = k A^T``, ``dE_j/dmu = 1``.

    Returns ``(dk [N_E, d*n_int], dmu, dt)`` with ``dE_j/dt = 2(cos K_jx + cos K_jy)``
    for the 2D dispersion.
    """
    K = line_momenta(alpha, k_int, q, dim, LD)
    ng = np.asarray(alpha).shape[0]
    t = LD(t)
    dK = np.zeros_like(K)
    for i in range(ng):
        blk = slice(i * dim, (i + 1) * dim)
        dK[:, blk] = np.asarray(dE)[:, i:i + 1] * (-2 * t * np.sin(K[:, blk]))
    A = kron_alpha(alpha, dim).astype(LD)
    dk_full = dK @ A
    n_k = np.asarray(k_int).shape[1]
    dt = LD(0)
    for i in range(ng):
        dt += np.sum(np.asarray(dE, dtype=LD)[:, i] * 2 * np.cos(K[:, i * dim:(i + 1) * dim]).sum(axis=1))
    return dk_full[:, :n_k], np.sum(np.asarray(dE, dtype=LD)), dt
