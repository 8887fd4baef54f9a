"""Helpers for GPU-vs-oracle parity tests (test infrastructure).

Error metric: at every (frequency, sample) point the absolute difference is
divided by ``sum_t |v_t|``, the sum of the magnitudes of the flat terms
computed by the oracle.  That is the scale of the rounding error of any
evaluation of the sum, so the bound holds whether or not the terms cancel.
Points within ``near`` of a pole of one term -- a Bose-type leaf argument
``|e.E| < near`` or a denominator ``|D| < near`` -- lose digits to the
rounding of their arguments in float64 on both sides of the comparison and are
held to the looser ``tol_near``.

The plain relative error ``|got - ref| / |ref|`` is held to the same ``tol``
wherever it is attainable: away from poles, at points whose cancellation ratio
``sum_t |v_t| / |ref|`` is at most ``COND_MAX``.  Beyond that ratio the terms
cancel to a total far below their own size (exponentially small totals, where
no float64 sum over terms is relatively accurate), and only the
condition-aware bound applies.
"""
from __future__ import annotations

import numpy as np

from oracle.construct import canonical, construct
from oracle.evaluate import evaluate_terms, energies_from_k, term_magnitudes

TOL = 1e-10        # relative to sum_t |v_t|, away from poles
TOL_NEAR = 1e-6    # within NEAR of a pole of one term
NEAR = 1e-4
COND_MAX = 1e4     # the plain relative bar applies up to this cancellation ratio


def oracle_terms(d):
    return canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))


def pole_distance(terms, n_int, E, w, e_reg=0.0):
    """min over Bose-type leaves of |e.E (+e_reg)| and over denominators of
    |D|, per (frequency, sample)."""
    E = np.asarray(E)
    E = E.astype(np.complex128 if np.iscomplexobj(E) else np.float64)
    w = np.asarray(w)
    if w.ndim == 1:
        w = w[:, None]
    dist = np.full((w.shape[0], E.shape[0]), np.inf)
    for _, leaves, dens in terms:
        for sigma, e in leaves:
            if sigma < 0:
                x = np.abs(E @ np.asarray(e, dtype=np.float64) + e_reg)   # |x| at complex E too
                dist = np.minimum(dist, x[None, :])
        for e, a in dens:
            base = E @ np.asarray(e, dtype=np.float64)
            ext = np.asarray(a[n_int:], dtype=np.float64)
            dd = np.abs(base[None, :] + (w @ ext)[:, None])
            dist = np.minimum(dist, dd)
    return dist


def reference(d, E, w, beta, e_reg=0.0, terms=None):
    terms = terms if terms is not None else oracle_terms(d)
    ref = evaluate_terms(terms, d.n_int, E, w, beta, e_reg).astype(np.complex128)
    scale = term_magnitudes(terms, d.n_int, E, w, beta, e_reg).astype(np.float64)
    dist = pole_distance(terms, d.n_int, E, w, e_reg)
    return ref, scale, dist


def reference_hubbard(d, k, q, t, mu, w, beta, e_reg=0.0, terms=None):
    E = energies_from_k(d.alpha, k, q, t, mu)
    ref, scale, dist = reference(d, E, w, beta, e_reg, terms)
    return ref, scale, dist, E.astype(np.float64)


def check(got, ref, scale, dist, tol=TOL, tol_near=TOL_NEAR, near=NEAR, label="", cond_max=COND_MAX,
          stats=None):
    """Assert the bars above; returns the worst condition-aware error away from
    poles.  ``stats``, a dict if given, receives the worst plain relative error
    where it is asserted, the number of such points, and percentiles of the
    cancellation ratio."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    diff = np.abs(got - ref)
    err = diff / np.maximum(scale, 1e-300)
    far = dist >= near
    assert np.all(np.isfinite(got[far])), f"{label}: non-finite output away from poles"
    worst = float(err[far].max()) if far.any() else 0.0
    assert worst <= tol, f"{label}: max error {worst:.3e} > {tol:.1e} (away from poles)"
    if (~far).any():
        worst_near = float(np.nanmax(err[~far]))
        assert worst_near <= tol_near, f"{label}: max error {worst_near:.3e} near poles"
    absref = np.abs(ref)
    ratio = scale / np.maximum(absref, 1e-300)
    plain = far & (ratio <= cond_max) & (absref > 0)   # cond_max = 0 turns the plain bar off
    worst_plain = float((diff[plain] / absref[plain]).max()) if plain.any() else 0.0
    assert worst_plain <= tol, (f"{label}: max plain relative error {worst_plain:.3e} > {tol:.1e} "
                                f"(away from poles, cancellation ratio <= {cond_max:.0e})")
    if stats is not None:
        r = ratio[far] if far.any() else np.zeros(1)
        stats.update({"worst_plain_rel": worst_plain, "plain_points": int(plain.sum()),
                      "far_points": int(far.sum()), "ratio_p50": float(np.percentile(r, 50)),
                      "ratio_p90": float(np.percentile(r, 90)), "ratio_p99": float(np.percentile(r, 99)),
                      "worst_scaled": worst})
    return worst


def far_from_poles(terms, n_int, E, w, e_reg=0.0, near=NEAR):
    """Indices of samples whose every Bose-type leaf argument and denominator
    stays at least ``near`` away from zero at every frequency row."""
    return np.nonzero(pole_distance(terms, n_int, E, w, e_reg).min(axis=0) >= near)[0]


def gradient_scale(terms, n_int, E, w, beta, cot, e_reg=0.0):
    """Per sample and energy, sum over terms of |dL_t/dE_i|: the rounding scale
    of the summed gradient (the analogue of sum_t |v_t| for values)."""
    return gradient_scales(terms, n_int, E, w, beta, cot, e_reg)["E"]


def gradient_scales(terms, n_int, E, w, beta, cot, e_reg=0.0, hubbard=None):
    """Rounding scales of every adjoint output: sums over terms (and over
    samples for the reduced outputs) of the magnitudes of the single-term
    contributions.  ``hubbard = (alpha, k, q, t, mu)`` adds the momentum path."""
    from oracle.evaluate import gradients, line_momenta
    E = np.asarray(E)
    out = {"E": np.zeros(E.shape, dtype=np.float64), "beta": 0.0, "w": 0.0}
    if hubbard is not None:
        alpha, k, q, t, mu = hubbard
        K = line_momenta(alpha, k, q).astype(np.float64)
        ng = np.asarray(alpha).shape[0]
        sin = np.sin(K)
        cs = np.stack([np.cos(K[:, 2 * j]) + np.cos(K[:, 2 * j + 1]) for j in range(ng)], axis=1)
        out.update({"k": np.zeros(np.asarray(k).shape), "mu": 0.0, "t": 0.0})
        A = np.kron(np.asarray(alpha, dtype=np.float64), np.eye(2))
    for term in terms:
        de, db, dw = gradients([term], n_int, E, w, beta, cot, e_reg, per_sample=True)
        de = de.astype(np.complex128 if np.iscomplexobj(de) else np.float64)
        out["E"] += np.abs(de)
        out["beta"] += float(np.sum(np.abs(db.astype(np.float64))))
        out["w"] += float(np.sum(np.abs(dw.astype(np.complex128))))
        if hubbard is not None:
            dK = np.repeat(de, 2, axis=1) * (-2 * t * sin)
            out["k"] += np.abs((dK @ A)[:, :np.asarray(k).shape[1]])
            out["mu"] += float(np.sum(np.abs(de.sum(axis=1))))
            out["t"] += float(np.sum(np.abs((de * 2 * cs).sum(axis=1))))
    return out
