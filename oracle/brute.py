"""Oracle: the plain definition Eq. (1) by truncated Matsubara sums.

``I = beta^-n sum_{nu_1..nu_n} prod_j 1/(sum_l alpha_jl w_l + sum_i eps_ji E_i)``
with ``w_l = i nu_l`` for the summed slots (Sec. 2.2, Eqs. (1)-(2)); the
energies may be complex.  Nothing
of the residue construction is used: the sums are done term by term over
``nu_m = (2m+1) pi / beta``, ``m = -M .. M-1`` (a range symmetric in ``nu``),
and the truncation error is removed by Richardson extrapolation in ``1/M``
over ``M, 2M, 4M, ...`` (the symmetric tail of a summand decaying like
``nu^-2`` is a power series in ``1/M``).

Works for up to three nested sums whose summands decay at least like
``nu^-2`` in every summed frequency (two or more propagators depending on it);
for a single propagator the symmetric sum and the residue result differ by
the convergence-factor term and the comparison is not made.
"""
from __future__ import annotations

import numpy as np


def _nu(m, beta):
    return (2.0 * m + 1.0) * np.pi / beta


def _richardson(values, ms, powers=(1, 2, 3, 4)):
    """Extrapolate S(M) = S + sum_k c_k M^-k to M -> infinity (least squares
    if there are more levels than unknowns)."""
    values = np.asarray(values)
    ms = np.asarray(ms, dtype=np.float64)
    p = [q for q in powers][: len(ms) - 1]
    A = np.ones((len(ms), 1 + len(p)))
    for j, q in enumerate(p):
        A[:, 1 + j] = ms ** (-float(q))
    sol_r = np.linalg.lstsq(A, values.real, rcond=None)[0]
    sol_i = np.linalg.lstsq(A, values.imag, rcond=None)[0]
    return sol_r[0] + 1j * sol_i[0]


def _denominators(alpha, eps, E, w_ext, n_int):
    """Constant parts c_j = eps_j.E + alpha_j,ext . w_ext and the summed
    coefficients alpha_j[:n_int]."""
    alpha = np.asarray(alpha, dtype=np.int64)
    eps = np.asarray(eps, dtype=np.int64)
    E = np.asarray(E)
    E = E.astype(np.complex128 if np.iscomplexobj(E) else np.float64)
    w_ext = np.atleast_1d(np.asarray(w_ext, dtype=np.complex128))
    c = eps @ E + alpha[:, n_int:] @ w_ext
    return alpha[:, :n_int].astype(np.float64), c


def single_sum(alpha, eps, E, w_ext, beta, M0=512, levels=5):
    """``beta^-1 sum_nu prod_j 1/(a_j i nu + c_j)`` for one summed slot."""
    a, c = _denominators(alpha, eps, E, w_ext, 1)
    vals, ms = [], []
    for k in range(levels):
        M = M0 * 2 ** k
        m = np.arange(-M, M)
        z = 1j * _nu(m, beta)
        h = np.ones_like(z)
        for j in range(len(c)):
            h = h / (a[j, 0] * z + c[j])
        vals.append(h.sum() / beta)
        ms.append(M)
    return _richardson(vals, ms)


def cube_sum(alpha, eps, E, w_ext, beta, n_int, M0, levels):
    """``beta^-n sum_{nu_1..nu_n} prod_j 1/(sum_p a_jp i nu_p + c_j)`` for
    ``n = 2`` or ``3``.

    When every set of summed frequencies is carried by more propagators than
    it has members the sum converges absolutely, so it is taken over growing
    cubes ``m_p in [-M, M)`` and extrapolated in ``1/M``.
    """
    a, c = _denominators(alpha, eps, E, w_ext, n_int)
    vals, ms = [], []
    for k in range(levels):
        M = M0 * 2 ** k
        m = np.arange(-M, M)
        z = 1j * _nu(m, beta)
        total = 0.0 + 0.0j
        if n_int == 2:
            for lo in range(0, len(m), 512):
                hi = min(lo + 512, len(m))
                h = np.ones((hi - lo, len(m)), dtype=np.complex128)
                for j in range(len(c)):
                    h = h / (a[j, 0] * z[lo:hi, None] + a[j, 1] * z[None, :] + c[j])
                total += h.sum()
        elif n_int == 3:
            for i0 in range(len(m)):
                h = np.ones((len(m), len(m)), dtype=np.complex128)
                for j in range(len(c)):
                    h = h / (a[j, 0] * z[i0] + a[j, 1] * z[:, None]
                             + a[j, 2] * z[None, :] + c[j])
                total += h.sum()
        else:
            raise ValueError("cube_sum handles two or three sums")
        vals.append(total / beta ** n_int)
        ms.append(M)
    return _richardson(vals, ms)


def brute_force(alpha, eps, n_int, E, w_ext, beta, **kw):
    """Eq. (1) at one energy vector and one external frequency vector."""
    if n_int == 0:
        a, c = _denominators(alpha, eps, E, w_ext, 0)
        return complex(np.prod(1.0 / c))
    if n_int == 1:
        return single_sum(alpha, eps, E, w_ext, beta, **kw)
    if n_int == 2:
        kw.setdefault("M0", 128)
        kw.setdefault("levels", 5)
        return cube_sum(alpha, eps, E, w_ext, beta, 2, **kw)
    if n_int == 3:
        kw.setdefault("M0", 16)
        kw.setdefault("levels", 4)
        return cube_sum(alpha, eps, E, w_ext, beta, 3, **kw)
    raise ValueError("brute force only for up to three sums")
