"""CPU pins of the library's Laplace quadrature (Sec. 2.2, Eq. (laplace)).

The quadrature is host code of the library, so it is checked here without a
GPU against what fixes it mathematically:
  * one term: the best rule in closed form;
  * the alternation theorem: the best n-term rule's relative error
    equioscillates at 2n + 1 points; an error curve that alternates with level
    ripples is therefore optimal (de la Vallee Poussin: no n-term rule does
    better than the smallest ripple);
  * uniqueness: an independent route (the oracle, scipy) reaches the same
    weights and exponents wherever both end with level ripples;
  * the returned error is the true maximum (a dense independent scan).
The ABI's argument checks run here too (they fail before any HIP call).
"""
import ctypes

import numpy as np
import pytest

from oracle import laplace as OL
from paper_2608_06536_amd import _lib

D = ctypes.POINTER(ctypes.c_double)


def lib_rule(n, x_min, x_max):
    w = (ctypes.c_double * n)()
    a = (ctypes.c_double * n)()
    e = ctypes.c_double()
    lev = ctypes.c_int32()
    st = _lib.lib().jk_laplace_quadrature(n, x_min, x_max, w, a, ctypes.byref(e),
                                          ctypes.byref(lev))
    assert st == _lib.JK_OK
    return np.array(w[:]), np.array(a[:]), e.value, bool(lev.value)


def scan_extrema(w, a, R, m=400001):
    """Independent dense scan: the maximum |eta| and the alternating extrema."""
    y = np.exp(np.linspace(0.0, np.log(R), m))
    e = OL.relative_error(w, a, y)
    idx = [0] + [i for i in range(1, m - 1) if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) < 0] + [m - 1]
    ext = []
    for i in idx:
        if ext and (ext[-1] > 0) == (e[i] > 0):
            if abs(e[i]) > abs(ext[-1]):
                ext[-1] = e[i]
        else:
            ext.append(e[i])
    return float(np.max(np.abs(e))), np.array(ext)


# (n, R) where the library's exchange ends with level ripples
LEVEL_CASES = [(1, 2.0), (1, 1e3), (2, 10.0), (3, 2.0), (4, 10.0), (4, 1e4), (6, 100.0),
               (8, 100.0), (8, 1e3), (10, 1e3), (10, 1e6), (12, 1e4)]


@pytest.mark.parametrize("R", [2.0, 10.0, 87.0, 1e4, 1e6])
def test_one_term_closed_form(R):
    w, a, E, lev = lib_rule(1, 1.0, R)
    w0, a0, E0 = OL.closed_form_one_term(R)
    assert lev
    assert abs(a[0] / a0 - 1) < 1e-10 and abs(w[0] / w0 - 1) < 1e-10
    assert abs(E / E0 - 1) < 1e-9
    wo, ao, Eo, levo = OL.minimax_rule(1, R)
    assert levo and abs(ao[0] / a0 - 1) < 1e-10 and abs(Eo / E0 - 1) < 1e-9


@pytest.mark.parametrize("n,R", LEVEL_CASES)
def test_rule_equioscillates(n, R):
    w, a, E, lev = lib_rule(n, 1.0, R)
    assert lev
    assert np.all(w > 0) and np.all(a > 0) and np.all(np.diff(a) > 0)
    mx, ext = scan_extrema(w, a, R)
    assert ext.size == 2 * n + 1
    assert np.all(np.sign(ext[1:]) != np.sign(ext[:-1]))
    mags = np.abs(ext)
    assert (mags.max() - mags.min()) <= 1e-4 * mags.max()     # level on the scan grid
    assert mx <= E * (1 + 1e-12)           # the reported error is the maximum
    assert mx >= E * (1 - 1e-4)


@pytest.mark.parametrize("n,R", [(2, 10.0), (4, 100.0), (6, 100.0), (8, 1e3), (10, 1e3),
                                 (12, 1e4)])
def test_rule_unique_two_routes(n, R):
    w, a, E, lev = lib_rule(n, 1.0, R)
    wo, ao, Eo, levo = OL.minimax_rule(n, R)
    assert lev and levo
    assert abs(E / Eo - 1) < 1e-7
    assert np.max(np.abs(w / wo - 1)) < 1e-6 and np.max(np.abs(a / ao - 1)) < 1e-6


def test_rule_scaling_and_monotone():
    # the rule for [x_min, x_max] is the [1, R] rule scaled by 1/x_min
    w1, a1, E1, _ = lib_rule(8, 1.0, 500.0)
    w2, a2, E2, _ = lib_rule(8, 0.25, 125.0)
    assert np.allclose(w2, 4.0 * w1, rtol=1e-13) and np.allclose(a2, 4.0 * a1, rtol=1e-13)
    assert E1 == E2
    # more terms: smaller error; wider range: larger error
    errs = [lib_rule(n, 1.0, 1e3)[2] for n in (4, 6, 8, 10, 12)]
    assert all(x > y for x, y in zip(errs, errs[1:]))
    errs = [lib_rule(8, 1.0, R)[2] for R in (100.0, 1e3, 1e4, 1e6)]
    assert all(x < y for x, y in zip(errs, errs[1:]))


def test_narrow_range_reports_honestly():
    # 10 terms on [1, 10]: the fit does not reach level ripples; it says so,
    # and its reported error is still the true maximum.
    w, a, E, lev = lib_rule(10, 1.0, 10.0)
    mx, _ = scan_extrema(w, a, 10.0)
    assert E < 1e-5
    assert mx <= E * (1 + 1e-12) and mx >= E * (1 - 1e-3)
    if not lev:
        assert E > 0


def test_ratio_below_two_widened():
    w, a, E, lev = lib_rule(3, 1.0, 1.5)
    w2, a2, E2, _ = lib_rule(3, 1.0, 2.0)
    assert np.array_equal(w, w2) and E == E2


@pytest.mark.parametrize("args", [(0, 1.0, 2.0), (21, 1.0, 2.0), (4, 0.0, 2.0), (4, -1.0, 2.0),
                                  (4, 2.0, 1.0), (4, 1.0, 2e9), (4, 1.0, float("inf")),
                                  (4, float("nan"), 2.0)])
def test_quadrature_invalid(args):
    n = max(args[0], 1)
    w = (ctypes.c_double * 32)()
    a = (ctypes.c_double * 32)()
    st = _lib.lib().jk_laplace_quadrature(args[0], args[1], args[2], w, a, None, None)
    assert st == _lib.JK_EINVAL
    assert n >= 1


# -------------------------------------------------------------- ABI checks
def _lp(**kw):
    d = dict(nao=10, naux=4, nocc=3, nvir=5, nvec=2, npts=4, precision=0, flags=3, nslice=0)
    d.update(kw)
    return _lib.LaplaceProblem(*[d[k] for k, _ in _lib.LaplaceProblem._fields_])


@pytest.mark.parametrize("bad", [dict(nao=0), dict(nocc=0), dict(nocc=11), dict(nvir=0),
                                 dict(nvec=0), dict(npts=0), dict(npts=21), dict(precision=5),
                                 dict(flags=8), dict(naux=0)])
def test_laplace_problem_invalid(bad):
    L = _lib.lib()
    p = _lp(**bad)
    assert L.jk_laplace_workspace_bytes(ctypes.byref(p)) == 0
    w = (ctypes.c_double * 32)(*([1.0] * 32))
    st = L.jk_laplace_build(ctypes.byref(p), 8, 8, 8, 8, 8, 8, w, w, 0.0, 8, 8, 256, 1 << 40, None)
    assert st == _lib.JK_EINVAL


def test_laplace_build_validation():
    L = _lib.lib()
    p = _lp()
    need = L.jk_laplace_workspace_bytes(ctypes.byref(p))
    assert need > 0 and need % 256 == 0
    w = (ctypes.c_double * 4)(1.0, 1.0, 1.0, 1.0)
    bad = (ctypes.c_double * 4)(1.0, float("nan"), 1.0, 1.0)
    args = [8, 8, 8, 8, 8, 8]
    assert L.jk_laplace_build(ctypes.byref(p), *args, w, w, 0.0, 8, 8, 256, need - 1,
                              None) == _lib.JK_EWORKSPACE
    assert L.jk_laplace_build(ctypes.byref(p), *args, w, w, 0.0, 8, 8, 264, need,
                              None) == _lib.JK_EINVAL
    assert L.jk_laplace_build(ctypes.byref(p), 8, 8, 8, 8, 8, None, w, w, 0.0, 8, 8, 256, need,
                              None) == _lib.JK_EINVAL
    assert L.jk_laplace_build(ctypes.byref(p), *args, w, bad, 0.0, 8, 8, 256, need,
                              None) == _lib.JK_EINVAL
    assert L.jk_laplace_build(ctypes.byref(p), *args, w, w, float("inf"), 8, 8, 256, need,
                              None) == _lib.JK_EINVAL
    pk = _lp(flags=2)
    assert L.jk_laplace_build(ctypes.byref(pk), *args, w, w, 0.0, 8, None, 256, need,
                              None) == _lib.JK_EINVAL


@pytest.mark.parametrize("args", [
    dict(nao=0), dict(norb=0), dict(rank=0), dict(nvec=0), dict(npts=0), dict(npts=21),
    dict(nao=20000), dict(X=None, rank=4),
])
def test_laplace_factors_invalid(args):
    L = _lib.lib()
    d = dict(nao=10, norb=5, rank=3, nvec=1, npts=2, X=8)
    d.update(args)
    a = (ctypes.c_double * 32)(*([1.0] * 32))
    st = L.jk_laplace_factors(d["nao"], d["norb"], d["rank"], d["nvec"], d["npts"], 8, 8, d["X"],
                              a, a, 1.0, 8, None)
    assert st == _lib.JK_EINVAL
