"""Python binding of the C ABI in include/jk.h (argument marshalling only).

PyTorch supplies device memory and the current HIP stream; every step of the
J/K path runs in the library's HIP kernels.

    J, K = jk_build(B, CL, CR)                  # Sec. 2.3, Eq. (4)
    F = jk_fock(B, CL, CR, 2.0, -a_x, B_lr, -b)  # 2J - a_x K - b K_lr in one call
    dB, dCL, dCR = jk_vjp(B, CL, CR, Jbar, Kbar) # Sec. 2.1, Eq. (1)
    J, K = jk(B, CL, CR)                        # differentiable (autograd)

Shapes: B [naux][nao][nao] (each slab symmetric), or packed upper triangles
B [naux][nao (nao + 1) / 2] (row by row, the order of numpy's triu_indices),
CL, CR [nd][nao][r], J, K, Jbar, Kbar [nd][nao][nao]; all float64,
contiguous, on the GPU.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

_PREC = {"fp64": _lib.JK_FP64, "mixed": _lib.JK_MIXED}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, name, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def make_problem(nao, naux, nd, r, precision="fp64", want_j=True, want_k=True, nslice=0,
                 packed=False):
    flags = (_lib.JK_WANT_J if want_j else 0) | (_lib.JK_WANT_K if want_k else 0)
    if flags == 0:
        raise ValueError("nothing requested")
    if packed:
        flags |= _lib.JK_B_PACKED
    return _lib.Problem(int(nao), int(naux), int(nd), int(r), int(_PREC[precision]), flags,
                        int(nslice), 0)


def workspace_bytes(prob) -> int:
    return int(_lib.lib().jk_workspace_bytes(ctypes.byref(prob)))


def _workspace(nbytes, device):
    # 256-byte alignment: the caching allocator hands out 512-byte aligned blocks.
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def is_packed(B, nao):
    """True for packed slabs [naux][nao (nao + 1) / 2], False for [naux][nao][nao]."""
    if B.dim() == 2 and B.shape[1] == nao * (nao + 1) // 2:
        return True
    if B.dim() == 3 and tuple(B.shape[1:]) == (nao, nao):
        return False
    raise ValueError(f"B must be [naux][{nao}][{nao}] or packed [naux][{nao * (nao + 1) // 2}]")


def _shapes(B, CL, CR):
    _check_tensor(B, "B")
    _check_tensor(CL, "CL")
    _check_tensor(CR, "CR")
    if CL.dim() != 3:
        raise ValueError("CL must be [nd][nao][r]")
    nao = CL.shape[1]
    is_packed(B, nao)
    naux = B.shape[0]
    if tuple(CR.shape) != tuple(CL.shape):
        raise ValueError("CR must have the shape of CL")
    return nao, naux, CL.shape[0], CL.shape[2]


def slice_b(B, nao, out=None):
    """Digit planes of B for the mixed precision (jk_slice_b), made once and
    passed to jk_build(..., precision="mixed", slices=...) for every build
    over the same B.  Returns a uint8 tensor on B's device."""
    _check_tensor(B, "B")
    packed = is_packed(B, nao)
    prob = make_problem(nao, B.shape[0], 1, 1, "mixed", packed=packed)
    n = int(_lib.lib().jk_slices_bytes(ctypes.byref(prob)))
    if n == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_slices_bytes")
    S = out if out is not None else _workspace(n, B.device)
    st = _lib.lib().jk_slice_b(ctypes.byref(prob), _ptr(B), _ptr(S), S.numel(), _stream())
    _lib.check(st, "jk_slice_b")
    return S


def jk_build(B, CL, CR, precision="fp64", want_j=True, want_k=True, nslice=0, out=None, ws=None,
             slices=None):
    """J_k = sum_Q <B^Q, D_k> B^Q and K_k = sum_Q B^Q D_k B^Q for D_k = CL_k CR_k^T.
    slices: B's digit planes from slice_b (precision "mixed" only)."""
    nao, naux, nd, r = _shapes(B, CL, CR)
    prob = make_problem(nao, naux, nd, r, precision, want_j, want_k, nslice, is_packed(B, nao))
    if out is None:
        J = torch.empty((nd, nao, nao), dtype=torch.float64, device=B.device) if want_j else None
        K = torch.empty((nd, nao, nao), dtype=torch.float64, device=B.device) if want_k else None
    else:
        J, K = out
    for t, name in ((J, "J"), (K, "K")):
        if t is not None:
            _check_tensor(t, name, (nd, nao, nao))
    nbytes = workspace_bytes(prob)
    if nbytes == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_build")
    if ws is None:
        ws = _workspace(nbytes, B.device)
    if slices is not None:
        st = _lib.lib().jk_build_sliced(ctypes.byref(prob), _ptr(B), _ptr(slices), slices.numel(),
                                        _ptr(CL), _ptr(CR), _ptr(J), _ptr(K), _ptr(ws), ws.numel(),
                                        _stream())
        _lib.check(st, "jk_build_sliced")
        return J, K
    st = _lib.lib().jk_build(ctypes.byref(prob), _ptr(B), _ptr(CL), _ptr(CR), _ptr(J), _ptr(K),
                             _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "jk_build")
    return J, K


def jk_fock(B, CL, CR, c_j=2.0, c_k=-1.0, B_lr=None, c_lr=0.0, precision="fp64", nslice=0,
            out=None, ws=None):
    """F_k = c_j J[D_k] + c_k K[D_k] + c_lr K_lr[D_k] in one call, K_lr from
    the second factor set B_lr [naux_lr][nao][nao] (or none)."""
    nao, naux, nd, r = _shapes(B, CL, CR)
    packed = is_packed(B, nao)
    naux_lr = 0
    if B_lr is not None:
        _check_tensor(B_lr, "B_lr")
        if is_packed(B_lr, nao) != packed:
            raise ValueError("B_lr must have the layout of B")
        naux_lr = B_lr.shape[0]
    prob = make_problem(nao, naux, nd, r, precision, True, True, nslice, packed)
    F = out if out is not None else torch.empty((nd, nao, nao), dtype=torch.float64,
                                                device=B.device)
    _check_tensor(F, "F", (nd, nao, nao))
    nbytes = int(_lib.lib().jk_fock_workspace_bytes(ctypes.byref(prob), naux_lr))
    if nbytes == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_fock")
    if ws is None:
        ws = _workspace(nbytes, B.device)
    coef = (ctypes.c_double * 3)(float(c_j), float(c_k), float(c_lr))
    st = _lib.lib().jk_fock(ctypes.byref(prob), _ptr(B), _ptr(B_lr), naux_lr, _ptr(CL), _ptr(CR),
                            coef, _ptr(F), _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "jk_fock")
    return F


def autotune(B, CL, CR, precision="fp64", reps=2, out=None, ws=None):
    """Times the candidate plans of this problem, records the fastest for its
    shape class (jk_tune.h) and returns (J, K, {"ht_tile", "chunk_mb"})."""
    nao, naux, nd, r = _shapes(B, CL, CR)
    prob = make_problem(nao, naux, nd, r, precision, packed=is_packed(B, nao))
    if out is None:
        J = torch.empty((nd, nao, nao), dtype=torch.float64, device=B.device)
        K = torch.empty_like(J)
    else:
        J, K = out
    if ws is None:
        ws = _workspace(workspace_bytes(prob), B.device)
    t = _lib.Tuning()
    st = _lib.lib().jk_autotune(ctypes.byref(prob), _ptr(B), _ptr(CL), _ptr(CR), _ptr(J), _ptr(K),
                                _ptr(ws), ws.numel(), _stream(), int(reps), ctypes.byref(t))
    _lib.check(st, "jk_autotune")
    return J, K, {"ht_tile": t.ht_tile, "chunk_mb": t.chunk_mb}


def autotune_batched(items, precision="fp64", reps=2):
    """Autotunes one member of each shape class present in a batch (the class
    of jk_tune.h: nao and ndens * rank in steps of 64); returns {class: plan}.
    jk_build_batched then builds every member with its class's plan."""
    done = {}
    for B, CL, CR in items:
        nao, R = CL.shape[1], CL.shape[0] * CL.shape[2]
        key = ((nao + 63) // 64, (R + 63) // 64)
        if key not in done:
            _, _, done[key] = autotune(B, CL, CR, precision, reps)
    return done


def tuning_get(prob):
    t = _lib.Tuning()
    _lib.check(_lib.lib().jk_tuning_get(ctypes.byref(prob), ctypes.byref(t)), "jk_tuning_get")
    return {"ht_tile": t.ht_tile, "chunk_mb": t.chunk_mb}


def tuning_set(prob, ht_tile, chunk_mb):
    t = _lib.Tuning(int(ht_tile), int(chunk_mb))
    _lib.check(_lib.lib().jk_tuning_set(ctypes.byref(prob), ctypes.byref(t)), "jk_tuning_set")


def plan_describe(prob, ht_tile=None, chunk_mb=None):
    """What the plan (the current one, or {ht_tile, chunk_mb}) does with the
    problem: slabs per chunk, exchange splits and, for the mixed precision,
    the deepest int32 slice sum against its exactness cap (host only)."""
    t = None
    if ht_tile is not None or chunk_mb is not None:
        cur = tuning_get(prob)
        t = _lib.Tuning(int(cur["ht_tile"] if ht_tile is None else ht_tile),
                        int(cur["chunk_mb"] if chunk_mb is None else chunk_mb))
    info = _lib.PlanInfo()
    _lib.check(_lib.lib().jk_plan_describe(ctypes.byref(prob), None if t is None else ctypes.byref(t),
                                           ctypes.byref(info)), "jk_plan_describe")
    return {f: getattr(info, f) for f, _ in _lib.PlanInfo._fields_ if f != "reserved"}


def tuning_clear():
    _lib.lib().jk_tuning_clear()


def tuning_save() -> str:
    n = int(_lib.lib().jk_tuning_save(None, 0))
    buf = ctypes.create_string_buffer(n)
    _lib.lib().jk_tuning_save(buf, n)
    return buf.value.decode()


def tuning_load(text: str):
    _lib.check(_lib.lib().jk_tuning_load(text.encode()), "jk_tuning_load")


def batched_workspace_bytes(probs) -> int:
    arr = (_lib.Problem * len(probs))(*probs)
    return int(_lib.lib().jk_batched_workspace_bytes(len(probs), arr))


def jk_build_batched(items, precision="fp64", want_j=True, want_k=True, nslice=0, outs=None,
                     ws=None):
    """items: list of (B, CL, CR) of uneven sizes; returns a list of (J, K)."""
    n = len(items)
    probs, res = [], []
    for g, (B, CL, CR) in enumerate(items):
        nao, naux, nd, r = _shapes(B, CL, CR)
        probs.append(make_problem(nao, naux, nd, r, precision, want_j, want_k, nslice,
                                  is_packed(B, nao)))
        if outs is None:
            J = torch.empty((nd, nao, nao), dtype=torch.float64, device=B.device) if want_j else None
            K = torch.empty((nd, nao, nao), dtype=torch.float64, device=B.device) if want_k else None
        else:
            J, K = outs[g]
        res.append((J, K))
    arr = (_lib.Problem * n)(*probs)
    VP = ctypes.c_void_p * n
    pb = VP(*[B.data_ptr() for B, _, _ in items])
    pl = VP(*[CL.data_ptr() for _, CL, _ in items])
    pr = VP(*[CR.data_ptr() for _, _, CR in items])
    pj = VP(*[(J.data_ptr() if J is not None else 0) for J, _ in res])
    pk = VP(*[(K.data_ptr() if K is not None else 0) for _, K in res])
    nbytes = batched_workspace_bytes(probs)
    if nbytes == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_build_batched")
    if ws is None:
        ws = _workspace(nbytes, items[0][0].device)
    st = _lib.lib().jk_build_batched(n, arr, pb, pl, pr, pj, pk, _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "jk_build_batched")
    return res


def jk_vjp(B, CL, CR, Jbar=None, Kbar=None, want_dB=True, want_dC=True, out=None, ws=None):
    """Adjoints (dB, dCL, dCR) of L = sum_k <Jbar_k, J_k> + <Kbar_k, K_k>."""
    nao, naux, nd, r = _shapes(B, CL, CR)
    for t, name in ((Jbar, "Jbar"), (Kbar, "Kbar")):
        if t is not None:
            _check_tensor(t, name, (nd, nao, nao))
    # packed slabs travel as a flag, so the library refuses them before any launch
    prob = make_problem(nao, naux, nd, r, "fp64", packed=is_packed(B, nao))
    if out is None:
        dB = torch.empty_like(B) if want_dB else None
        dCL = torch.empty_like(CL) if want_dC else None
        dCR = torch.empty_like(CR) if want_dC else None
    else:
        dB, dCL, dCR = out
    nbytes = workspace_bytes(prob)
    if nbytes == 0:
        raise _lib.JKError(_lib.JK_EINVAL, "jk_vjp")
    if ws is None:
        ws = _workspace(nbytes, B.device)
    st = _lib.lib().jk_vjp(ctypes.byref(prob), _ptr(B), _ptr(CL), _ptr(CR), _ptr(Jbar), _ptr(Kbar),
                           _ptr(dB), _ptr(dCL), _ptr(dCR), _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "jk_vjp")
    return dB, dCL, dCR


class JKFunction(torch.autograd.Function):
    """(B, CL, CR) -> (J, K) with the reverse pass through jk_vjp."""

    @staticmethod
    def forward(ctx, B, CL, CR, precision="fp64"):
        J, K = jk_build(B.contiguous(), CL.contiguous(), CR.contiguous(), precision)
        ctx.save_for_backward(B, CL, CR)
        return J, K

    @staticmethod
    def backward(ctx, Jbar, Kbar):
        B, CL, CR = ctx.saved_tensors
        Jbar = None if Jbar is None else Jbar.contiguous()
        Kbar = None if Kbar is None else Kbar.contiguous()
        need_b = ctx.needs_input_grad[0]
        need_c = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        dB, dCL, dCR = jk_vjp(B.contiguous(), CL.contiguous(), CR.contiguous(), Jbar, Kbar,
                              want_dB=need_b, want_dC=need_c)
        return dB, dCL, dCR, None


def jk(B, CL, CR, precision="fp64"):
    return JKFunction.apply(B, CL, CR, precision)
