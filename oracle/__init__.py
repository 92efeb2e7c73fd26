"""ctypes binding of the FP64 CPU oracle (``jk_oracle.c``).

TEST INFRASTRUCTURE ONLY: the independent reference that the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library never imports, links or calls it.

Every function takes and returns C-contiguous float64 numpy arrays in the
layouts documented in ``jk_oracle.c``:
``B[naux][nao][nao]``, ``CL, CR[nd][nao][r]``, ``D, J, K, W, V[nd][nao][nao]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jk_oracle.c")
_LIB = os.path.join(_HERE, "libjkoracle.so")
_lib = None

_P = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int64
_IP = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        for name, nargs in [("jko_eri4", 0), ("jko_jk_from_eri", 0), ("jko_density", 0),
                            ("jko_project", 0), ("jko_coulomb", 0), ("jko_exchange", 0),
                            ("jko_jk_factored", 0), ("jko_jk_entries", 0), ("jko_vjp", 0),
                            ("jko_db_entries", 0), ("jko_jvp", 0), ("jko_dc_density", 0),
                            ("jko_vjp_factored", 0)]:
            getattr(lib, name).restype = None
        lib.jko_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_IP)


def num_threads() -> int:
    return int(_load().jko_num_threads())


def eri4(B):
    """T0: (mn|ls) = sum_Q B^Q_mn B^Q_ls, shape [nao][nao][nao][nao]."""
    B = _c(B)
    naux, nao, _ = B.shape
    eri = np.empty((nao, nao, nao, nao))
    _load().jko_eri4(_I(nao), _I(naux), _d(B), _d(eri))
    return eri


def jk_from_eri(eri, D):
    """T0: J_mn = sum_ls (mn|ls) D_ls, K_mn = sum_ls (ml|sn) D_ls, one density."""
    eri, D = _c(eri), _c(D)
    nao = D.shape[0]
    J = np.empty((nao, nao))
    K = np.empty((nao, nao))
    _load().jko_jk_from_eri(_I(nao), _d(eri), _d(D), _d(J), _d(K))
    return J, K


def density(CL, CR):
    CL, CR = _c(CL), _c(CR)
    nd, nao, r = CL.shape
    D = np.empty((nd, nao, nao))
    _load().jko_density(_I(nd), _I(nao), _I(r), _d(CL), _d(CR), _d(D))
    return D


def project(B, A):
    """g[k][Q] = <A_k, B^Q>."""
    B, A = _c(B), _c(A)
    naux, nao, _ = B.shape
    nd = A.shape[0]
    g = np.empty((nd, naux))
    _load().jko_project(_I(nd), _I(nao), _I(naux), _d(B), _d(A), _d(g))
    return g


def coulomb(B, g):
    """J_k = sum_Q g[k][Q] B^Q."""
    B, g = _c(B), _c(g)
    naux, nao, _ = B.shape
    nd = g.shape[0]
    J = np.empty((nd, nao, nao))
    _load().jko_coulomb(_I(nd), _I(nao), _I(naux), _d(B), _d(g), _d(J))
    return J


def exchange(B, D):
    """K_k = sum_Q B^Q D_k B^Q (literal products, general B)."""
    B, D = _c(B), _c(D)
    naux, nao, _ = B.shape
    nd = D.shape[0]
    K = np.empty((nd, nao, nao))
    _load().jko_exchange(_I(nd), _I(nao), _I(naux), _d(B), _d(D), _d(K))
    return K


def jk_plain(B, CL, CR):
    """T1: explicit D, gamma = <D, B^Q>, J = sum gamma B, K = sum B D B."""
    D = density(CL, CR)
    g = project(B, D)
    return coulomb(B, g), exchange(B, D)


def jk_from_density(B, D):
    """T1 on explicit (possibly non-factored) densities D[nd][nao][nao]."""
    g = project(B, D)
    return coulomb(B, g), exchange(B, D)


def jk_factored(B, CL, CR):
    """T2: half-transform form (symmetric B).  Returns (J, K, gamma)."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    naux, nao, _ = B.shape
    nd, _, r = CL.shape
    J = np.empty((nd, nao, nao))
    K = np.empty((nd, nao, nao))
    g = np.empty((nd, naux))
    _load().jko_jk_factored(_I(nd), _I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR),
                            _d(J), _d(K), _d(g))
    return J, K, g


def jk_entries(B, CL, CR, ks, ms, ns):
    """T3: entries J[k][m][n], K[k][m][n] computed one by one (symmetric B);
    gamma from the plain projection <D_k, B^Q>."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    naux, nao, _ = B.shape
    r = CL.shape[2]
    gam = project(B, density(CL, CR))
    ks, pk = _i(ks)
    ms, pm = _i(ms)
    ns, pn = _i(ns)
    n = ks.size
    Jo = np.empty(n)
    Ko = np.empty(n)
    _load().jko_jk_entries(_I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR), _d(gam), _I(n),
                           pk, pm, pn, _d(Jo), _d(Ko))
    return Jo, Ko


def vjp(B, CL, CR, W=None, V=None, want_dB=True):
    """Reverse-mode derivative of sum_k <W_k,J_k> + <V_k,K_k> (general B).
    Returns (dB or None, dCL, dCR)."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    W = None if W is None else _c(W)
    V = None if V is None else _c(V)
    naux, nao, _ = B.shape
    nd, _, r = CL.shape
    dB = np.empty_like(B) if want_dB else None
    dCL = np.empty_like(CL)
    dCR = np.empty_like(CR)
    _load().jko_vjp(_I(nd), _I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR), _d(W), _d(V),
                    _d(dB), _d(dCL), _d(dCR))
    return dB, dCL, dCR


def jvp(B, CL, CR, dB=None, dCL=None, dCR=None):
    """Forward-mode derivative (dJ, dK) along (dB, dCL, dCR) (general B)."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    dB = None if dB is None else _c(dB)
    dCL = None if dCL is None else _c(dCL)
    dCR = None if dCR is None else _c(dCR)
    naux, nao, _ = B.shape
    nd, _, r = CL.shape
    dJ = np.empty((nd, nao, nao))
    dK = np.empty((nd, nao, nao))
    _load().jko_jvp(_I(nd), _I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR), _d(dB),
                    _d(dCL), _d(dCR), _d(dJ), _d(dK))
    return dJ, dK


def vjp_factored(B, CL, CR, W=None, V=None, q0=0, q1=None, want_dB=True, want_dCL=True,
                 want_dCR=True):
    """Factored derivative (symmetric B) over slabs [q0, q1).  Returns
    (dB or None, dCL or None, dCR or None); dB rows outside [q0, q1) are zero."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    W = None if W is None else _c(W)
    V = None if V is None else _c(V)
    naux, nao, _ = B.shape
    nd, _, r = CL.shape
    q1 = naux if q1 is None else q1
    dB = np.zeros_like(B) if want_dB else None
    dCL = np.empty_like(CL) if want_dCL else None
    dCR = np.empty_like(CR) if want_dCR else None
    _load().jko_vjp_factored(_I(nd), _I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR), _d(W),
                             _d(V), _I(q0), _I(q1), _d(dB), _d(dCL), _d(dCR))
    return dB, dCL, dCR


def db_entries(B, CL, CR, W, V, qs, as_, bs):
    """Entries dB[Q][a][b] one by one (symmetric B)."""
    B, CL, CR = _c(B), _c(CL), _c(CR)
    W = None if W is None else _c(W)
    V = None if V is None else _c(V)
    naux, nao, _ = B.shape
    nd, _, r = CL.shape
    qs, pq = _i(qs)
    as_, pa = _i(as_)
    bs, pb = _i(bs)
    out = np.empty(qs.size)
    _load().jko_db_entries(_I(nd), _I(nao), _I(naux), _I(r), _d(B), _d(CL), _d(CR), _d(W),
                           _d(V), _I(qs.size), pq, pa, pb, _d(out))
    return out


def dc_density(B, CLk, CRk, Wk, Vk):
    """dC_L, dC_R of one density (symmetric B), Q-outer."""
    B, CLk, CRk = _c(B), _c(CLk), _c(CRk)
    Wk = None if Wk is None else _c(Wk)
    Vk = None if Vk is None else _c(Vk)
    naux, nao, _ = B.shape
    r = CLk.shape[1]
    dl = np.empty((nao, r))
    dr = np.empty((nao, r))
    _load().jko_dc_density(_I(nao), _I(naux), _I(r), _d(B), _d(CLk), _d(CRk), _d(Wk), _d(Vk),
                           _d(dl), _d(dr))
    return dl, dr
