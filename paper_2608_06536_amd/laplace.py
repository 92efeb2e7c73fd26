"""Python binding of include/jk_laplace.h (argument marshalling only).

Sec. 2.2, Eq. (laplace): orbital-energy denominators as short exponential
sums, so that every denominator-weighted density is a set of ordinary
densities built from energy-scaled coefficients, each one J/K build.

    w, alpha, err, is_minimax = laplace_quadrature(8, x_min, x_max)
    CL = laplace_factors(C, e, alpha, coef, scale=+1.0)          # [npts][1][nao][norb]
    J, K, rule = laplace_jk(B, Cocc, e_occ, Cvir, e_vir, X)      # [npts][nvec][nao][nao]

The rule is computed on the host by the library; factors and builds run in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .jk import _PREC, _check_tensor, _ptr, _stream, _workspace, is_packed

__all__ = ["laplace_quadrature", "denominator_range", "laplace_factors", "laplace_jk"]


def laplace_quadrature(npts: int, x_min: float, x_max: float):
    """(w, alpha, max_rel_err, is_minimax): 1/x ~ sum_k w_k exp(-alpha_k x)
    on [x_min, x_max]; max_rel_err is measured on the returned rule."""
    w = (ctypes.c_double * int(npts))()
    a = (ctypes.c_double * int(npts))()
    err = ctypes.c_double()
    lev = ctypes.c_int32()
    st = _lib.lib().jk_laplace_quadrature(int(npts), float(x_min), float(x_max), w, a,
                                          ctypes.byref(err), ctypes.byref(lev))
    _lib.check(st, "jk_laplace_quadrature")
    return np.array(w[:]), np.array(a[:]), float(err.value), bool(lev.value)


def denominator_range(e_occ, e_vir, shift=0.0, excitations=2):
    """[x_min, x_max] of sum over `excitations` pairs of (e_a - e_i), plus
    shift, from host copies of the orbital energies."""
    eo = np.asarray(e_occ.detach().cpu() if isinstance(e_occ, torch.Tensor) else e_occ, float)
    ev = np.asarray(e_vir.detach().cpu() if isinstance(e_vir, torch.Tensor) else e_vir, float)
    lo = excitations * (ev.min() - eo.max()) + shift
    hi = excitations * (ev.max() - eo.min()) + shift
    if not lo > 0.0:
        raise ValueError(f"denominators must be positive (smallest is {lo})")
    return float(lo), float(hi)


def laplace_factors(C, e, alpha, coef, scale, X=None, nvec=1, out=None):
    """out[k][m] = coef_k C diag(exp(scale alpha_k e)) X_m^T (X None: no
    contraction, rank = norb, copied for each of nvec).  Returns
    [npts][nvec][nao][rank]."""
    _check_tensor(C, "C")
    _check_tensor(e, "e")
    if C.dim() != 2 or e.dim() != 1 or e.shape[0] != C.shape[1]:
        raise ValueError("C must be [nao][norb] and e [norb]")
    nao, norb = C.shape
    if X is not None:
        _check_tensor(X, "X")
        if X.dim() != 3 or X.shape[2] != norb:
            raise ValueError("X must be [nvec][rank][norb]")
        nvec, rank = X.shape[0], X.shape[1]
    else:
        rank = norb
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    npts = alpha.size
    if coef.size != npts:
        raise ValueError("alpha and coef must have the same length")
    if out is None:
        out = torch.empty((npts, nvec, nao, rank), dtype=torch.float64, device=C.device)
    _check_tensor(out, "out", (npts, nvec, nao, rank))
    dp = ctypes.POINTER(ctypes.c_double)
    st = _lib.lib().jk_laplace_factors(nao, norb, rank, nvec, npts, _ptr(C), _ptr(e), _ptr(X),
                                       alpha.ctypes.data_as(dp), coef.ctypes.data_as(dp),
                                       float(scale), _ptr(out), _stream())
    _lib.check(st, "jk_laplace_factors")
    return out


def make_laplace_problem(nao, naux, nocc, nvir, nvec, npts, precision="fp64", want_j=True,
                         want_k=True, nslice=0, packed=False):
    flags = (_lib.JK_WANT_J if want_j else 0) | (_lib.JK_WANT_K if want_k else 0)
    if flags == 0:
        raise ValueError("nothing requested")
    if packed:
        flags |= _lib.JK_B_PACKED
    return _lib.LaplaceProblem(int(nao), int(naux), int(nocc), int(nvir), int(nvec), int(npts),
                               int(_PREC[precision]), flags, int(nslice))


def laplace_jk(B, Cocc, e_occ, Cvir, e_vir, X, npts=8, shift=0.0, excitations=2, rule=None,
               precision="fp64", want_j=True, want_k=True, nslice=0, out=None, ws=None):
    """J and K of the transition pseudo-densities
    D_km = w_k exp(-alpha_k shift) Cocc e^{+alpha_k e_occ} X_m e^{-alpha_k e_vir} Cvir^T.

    rule: (w, alpha) to use; by default the library's rule for the range of
    `excitations` pairs of orbital-energy differences plus shift.  Returns
    (J, K, rule) with J, K of shape [npts][nvec][nao][nao] and rule =
    (w, alpha, max_rel_err, is_minimax) (err and flag None for a given rule).
    """
    for t, name in ((B, "B"), (Cocc, "Cocc"), (e_occ, "e_occ"), (Cvir, "Cvir"), (e_vir, "e_vir"),
                    (X, "X")):
        _check_tensor(t, name)
    nao, naux = Cocc.shape[0], B.shape[0]
    packed = is_packed(B, nao)
    nocc, nvir = Cocc.shape[1], Cvir.shape[1]
    if X.dim() != 3 or tuple(X.shape[1:]) != (nocc, nvir):
        raise ValueError("X must be [nvec][nocc][nvir]")
    nvec = X.shape[0]
    if rule is None:
        x_min, x_max = denominator_range(e_occ, e_vir, shift, excitations)
        w, alpha, err, lev = laplace_quadrature(npts, x_min, x_max)
    else:
        w, alpha = (np.ascontiguousarray(v, dtype=np.float64) for v in rule[:2])
        err = lev = None
    npts = w.size
    prob = make_laplace_problem(nao, naux, nocc, nvir, nvec, npts, precision, want_j, want_k,
                                nslice, packed)
    nbytes = int(_lib.lib().jk_laplace_workspace_bytes(ctypes.byref(prob)))
    if nbytes == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_laplace_build")
    shape = (npts, nvec, nao, nao)
    if out is None:
        J = torch.empty(shape, dtype=torch.float64, device=B.device) if want_j else None
        K = torch.empty(shape, dtype=torch.float64, device=B.device) if want_k else None
    else:
        J, K = out
    for t, name in ((J, "J"), (K, "K")):
        if t is not None:
            _check_tensor(t, name, shape)
    if ws is None:
        ws = _workspace(nbytes, B.device)
    dp = ctypes.POINTER(ctypes.c_double)
    w = np.ascontiguousarray(w, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    st = _lib.lib().jk_laplace_build(ctypes.byref(prob), _ptr(B), _ptr(Cocc), _ptr(e_occ),
                                     _ptr(Cvir), _ptr(e_vir), _ptr(X), w.ctypes.data_as(dp),
                                     alpha.ctypes.data_as(dp), float(shift), _ptr(J), _ptr(K),
                                     _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "jk_laplace_build")
    return J, K, (w, alpha, err, lev)
