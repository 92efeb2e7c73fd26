"""Oracle of the Laplace pseudo-density driver (Sec. 2.2, Eq. (laplace)).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library's Laplace
entry points are checked against.  Only the tests, the smoke check and the
benchmark's CPU baseline use it; the library never imports or calls it.

Plain numpy / scipy in FP64, small sizes:

* ``minimax_rule(n, R)`` -- the n-term exponential sum that minimizes the
  maximum relative error of 1/y on [1, R], reached by its own route
  (scipy's MINPACK Levenberg-Marquardt on least p-th powers from a
  trapezoid start, then Remez exchange with scipy's hybrid Newton solver).
  The best approximation is unique, so wherever two routes both end with
  level ripples they must agree.
* ``scaled_factors`` -- the energy-scaled factors
  ``coef_k C diag(exp(scale alpha_k e)) [X_m^T]``, written out.
* ``mo_eri`` -- MO integrals ``(pq|rs) = sum_Q (Cp^T B^Q Cq)_pq (Cr^T B^Q Cs)_rs``.
* ``pair_contraction`` / ``doubles_contraction`` -- the denominator-weighted
  contractions the pseudo-densities stand for, with the exact denominators
  or with a quadrature ``1/x ~ sum_k w_k exp(-alpha_k x)``:
      pair:     sJ_ia = sum_jb (ia|jb) X_jb / (e_b - e_j + shift)
                sK_ia = sum_jb (ij|ab) X_jb / (e_b - e_j + shift)
      doubles:  the same with denominators e_a + e_b - e_i - e_j + shift
  plus the bound ``sum_jb |(..)(..) X_jb| / x`` that a rule of maximum
  relative error E multiplies into an error bound.
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import optimize

__all__ = ["relative_error", "minimax_rule", "closed_form_one_term", "scaled_factors",
           "mo_eri", "pair_contraction", "doubles_contraction", "quadrature_of"]


# ------------------------------------------------------------------ the rule
def relative_error(w, a, y):
    """eta(y) = 1 - y sum_k w_k exp(-a_k y)."""
    y = np.asarray(y, dtype=float)
    return 1.0 - y * (np.exp(-np.outer(y, a)) @ np.asarray(w, dtype=float))


def closed_form_one_term(R):
    """The best one-term rule on [1, R] in closed form: y w exp(-a y) peaks at
    y = 1/a inside the range, so the error alternates at 1, 1/a, R with equal
    values at the ends, w exp(-a) = R w exp(-a R), which fixes
    a = ln R / (R - 1); equal magnitude at the peak, w/(a e) - 1 = 1 - w e^-a,
    fixes w.  Returns (w, a, E)."""
    a = np.log(R) / (R - 1.0)
    w = 2.0 / (1.0 / (a * np.e) + np.exp(-a))
    return w, a, w / (a * np.e) - 1.0


def _scan(w, a, R, m=40001):
    y = np.exp(np.linspace(0.0, np.log(R), m))
    return y, relative_error(w, a, y)


def _extrema(w, a, R):
    """Alternating local extrema of eta on [1, R] (ends included), refined."""
    y, e = _scan(w, a, R)
    pts = [(y[0], e[0])]
    for i in range(1, y.size - 1):
        if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) < 0:
            sg = 1.0 if e[i] > 0 else -1.0
            res = optimize.minimize_scalar(lambda t: -sg * relative_error(w, a, [np.exp(t)])[0],
                                           bounds=(np.log(y[i - 1]), np.log(y[i + 1])),
                                           method="bounded", options={"xatol": 1e-14})
            yv = float(np.exp(res.x))
            ev = float(relative_error(w, a, [yv])[0])
            pts.append((yv, ev) if sg * ev >= sg * e[i] else (y[i], e[i]))
    pts.append((y[-1], e[-1]))
    out = []
    for yv, ev in pts:
        if out and (out[-1][1] > 0) == (ev > 0):
            if abs(ev) > abs(out[-1][1]):
                out[-1] = (yv, ev)
        else:
            out.append((yv, ev))
    ys = np.array([p[0] for p in out])
    es = np.array([p[1] for p in out])
    return ys, es, max(np.max(np.abs(e)), np.max(np.abs(es)))


@functools.lru_cache(maxsize=64)
def minimax_rule(n: int, R: float):
    """(w, a, E, level) for the n-term rule on [1, R]; E is the measured
    maximum relative error, level whether the ripples came out level."""
    # trapezoid start for 1/y = int exp(s - y e^s) ds
    s_lo, s_hi = -np.log(R) - 2.5, 1.5 + 0.25 * np.log(n)
    s = np.linspace(s_lo, s_hi, n) if n > 1 else np.array([0.5 * (s_lo + s_hi)])
    h = (s_hi - s_lo) / max(n - 1, 1)
    p = np.concatenate([np.log(h) + s, s])            # (ln w, ln a)
    yg = np.exp(np.linspace(0.0, np.log(R), 24 * n + 48))
    for pw in (2, 4, 8, 16, 32, 64):
        sc = np.max(np.abs(relative_error(np.exp(p[:n]), np.exp(p[n:]), yg)))
        q = 0.5 * (pw - 2)

        def res(pp):
            e = relative_error(np.exp(pp[:n]), np.exp(pp[n:]), yg)
            return e * np.abs(e / sc) ** q

        with np.errstate(over="ignore", invalid="ignore"):
            p = optimize.least_squares(res, p, method="lm", max_nfev=300 * (2 * n + 1)).x
    w, a = np.exp(p[:n]), np.exp(p[n:])
    o = np.argsort(a)
    w, a = w[o], a[o]
    ys, es, E = _extrema(w, a, R)
    best = (w, a, E)
    level = False
    for _ in range(50):
        if ys.size != 2 * n + 1:
            break
        mags = np.abs(es)
        if mags.max() - mags.min() <= 1e-7 * mags.max():
            level = True
            break
        sgn = (-1.0) ** np.arange(2 * n + 1)

        def eqs(z):
            return relative_error(np.exp(z[:n]), np.exp(z[n:2 * n]), ys) - sgn * z[2 * n]

        z0 = np.concatenate([np.log(w), np.log(a), [es[0]]])
        sol = optimize.root(eqs, z0, method="hybr", options={"xtol": 1e-15})
        if not np.all(np.isfinite(sol.x)):
            break
        w, a = np.exp(sol.x[:n]), np.exp(sol.x[n:2 * n])
        o = np.argsort(a)
        w, a = w[o], a[o]
        ys, es, E = _extrema(w, a, R)
        if E < best[2]:
            best = (w, a, E)
    return best[0], best[1], best[2], level


def quadrature_of(w, alpha, x):
    """sum_k w_k exp(-alpha_k x), elementwise over the array x."""
    x = np.asarray(x, dtype=float)
    return np.tensordot(np.exp(-np.multiply.outer(x, alpha)), w, axes=([-1], [0]))


# --------------------------------------------------------------- the factors
def scaled_factors(C, e, alpha, coef, scale, X=None, nvec=1):
    """out[k][m] = coef_k C diag(exp(scale alpha_k e)) X_m^T (X None: no
    contraction, the same for every m).  Shape [npts][nvec][nao][rank]."""
    out = []
    for k in range(len(alpha)):
        Ck = coef[k] * C * np.exp(scale * alpha[k] * e)[None, :]
        if X is None:
            out.append(np.stack([Ck] * nvec))
        else:
            out.append(np.stack([Ck @ X[m].T for m in range(X.shape[0])]))
    return np.ascontiguousarray(np.stack(out))


# ---------------------------------------------------- MO-space definitions
def mo_eri(B, Cp, Cq, Cr, Cs):
    """(pq|rs) from the Cholesky vectors, [p][q][r][s]."""
    T1 = np.einsum("mp,Qmn,nq->Qpq", Cp, B, Cq)
    T2 = np.einsum("mr,Qmn,ns->Qrs", Cr, B, Cs)
    return np.einsum("Qpq,Qrs->pqrs", T1, T2)


def _integrals(B, Co, Cv):
    iajb = mo_eri(B, Co, Cv, Co, Cv)     # (ia|jb)
    ijab = mo_eri(B, Co, Co, Cv, Cv)     # (ij|ab)
    return iajb, np.transpose(ijab, (0, 2, 1, 3))   # -> [i][a][j][b]


def pair_contraction(B, Co, eo, Cv, ev, X, shift=0.0, rule=None):
    """(sJ, sK, bJ, bK) of the one-excitation denominator e_b - e_j + shift,
    exact (rule None) or with rule = (w, alpha)."""
    iajb, ijab = _integrals(B, Co, Cv)
    x = ev[None, :] - eo[:, None] + shift                      # [j][b]
    f = 1.0 / x if rule is None else quadrature_of(rule[0], rule[1], x)
    Y = X * f
    sJ = np.einsum("iajb,jb->ia", iajb, Y)
    sK = np.einsum("iajb,jb->ia", ijab, Y)
    bJ = np.einsum("iajb,jb->ia", np.abs(iajb), np.abs(X) / x)
    bK = np.einsum("iajb,jb->ia", np.abs(ijab), np.abs(X) / x)
    return sJ, sK, bJ, bK


def doubles_contraction(B, Co, eo, Cv, ev, X, shift=0.0, rule=None):
    """(sJ, sK, bJ, bK) of the denominator e_a + e_b - e_i - e_j + shift."""
    iajb, ijab = _integrals(B, Co, Cv)
    d = ev[None, :] - eo[:, None]
    x = d[:, :, None, None] + d[None, None, :, :] + shift       # [i][a][j][b]
    f = 1.0 / x if rule is None else quadrature_of(rule[0], rule[1], x)
    sJ = np.einsum("iajb,jb->ia", iajb * f, X)
    sK = np.einsum("iajb,jb->ia", ijab * f, X)
    bJ = np.einsum("iajb,jb->ia", np.abs(iajb) / x, np.abs(X))
    bK = np.einsum("iajb,jb->ia", np.abs(ijab) / x, np.abs(X))
    return sJ, sK, bJ, bK
