"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before any launch (no GPU needed: every
call here fails validation, so nothing is enqueued)."""
import ctypes
import os
import re

import pytest

from paper_2608_06536_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:[a-z_0-9]+\s+\*?)+(jk_[a-z_]+)\s*\(", txt, re.M)))


def test_header_symbols_exported():
    L = _lib.lib()
    names = _declared("jk.h")
    assert set(names) == set(_lib.EXPORTS)
    prof = _declared("jk_prof.h")
    assert set(prof) == set(_lib.PROF_EXPORTS)
    lap = _declared("jk_laplace.h")
    assert set(lap) == set(_lib.LAPLACE_EXPORTS)
    tune = _declared("jk_tune.h")
    assert set(tune) == set(_lib.TUNE_EXPORTS)
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["jk.h", "jk_laplace.h", "jk_prof.h",
                                                                "jk_tune.h"]
    for n in names + prof + lap + tune:
        assert hasattr(L, n), n


def _prob(**kw):
    d = dict(nao=10, naux=4, ndens=2, rank=3, precision=0, flags=3, nslice=0, reserved=0)
    d.update(kw)
    return _lib.Problem(*[d[k] for k, _ in _lib.Problem._fields_])


@pytest.mark.parametrize("bad", [
    dict(nao=0), dict(naux=0), dict(ndens=0), dict(rank=0), dict(rank=11), dict(precision=7),
    dict(flags=8), dict(flags=-1), dict(reserved=1), dict(precision=1, nslice=-1),
    dict(precision=1, nslice=9), dict(nao=1 << 20),
])
def test_invalid_problem(bad):
    L = _lib.lib()
    p = _prob(**bad)
    assert L.jk_workspace_bytes(ctypes.byref(p)) == 0
    st = L.jk_build(ctypes.byref(p), 8, 8, 8, 8, 8, 256, 1 << 40, None)
    assert st == _lib.JK_EINVAL
    st = L.jk_vjp(ctypes.byref(p), 8, 8, 8, 8, 8, 8, 8, 8, 256, 1 << 40, None)
    assert st == _lib.JK_EINVAL


def test_workspace_query_and_errors():
    L = _lib.lib()
    p = _prob()
    need = L.jk_workspace_bytes(ctypes.byref(p))
    assert need > 0 and need % 256 == 0
    # null required pointers
    assert L.jk_build(ctypes.byref(p), None, 8, 8, 8, 8, 256, need, None) == _lib.JK_EINVAL
    assert L.jk_build(ctypes.byref(p), 8, 8, 8, None, 8, 256, need, None) == _lib.JK_EINVAL
    # K not requested: K may be NULL, but ws too small still reported
    pj = _prob(flags=1)
    assert L.jk_build(ctypes.byref(pj), 8, 8, 8, 8, None, 256, 16, None) == _lib.JK_EWORKSPACE
    # misaligned workspace
    assert L.jk_build(ctypes.byref(p), 8, 8, 8, 8, 8, 264, need, None) == _lib.JK_EINVAL
    # too small workspace
    assert L.jk_build(ctypes.byref(p), 8, 8, 8, 8, 8, 256, need - 1, None) == _lib.JK_EWORKSPACE
    assert L.jk_vjp(ctypes.byref(p), 8, 8, 8, 8, 8, 8, 8, 8, 256, need - 1, None) == _lib.JK_EWORKSPACE
    # null problem
    assert L.jk_workspace_bytes(None) == 0
    assert L.jk_build(None, 8, 8, 8, 8, 8, 256, need, None) == _lib.JK_EINVAL


def test_batched_validation():
    L = _lib.lib()
    arr = (_lib.Problem * 2)(_prob(), _prob(nao=20))
    need = L.jk_batched_workspace_bytes(2, arr)
    assert need >= L.jk_workspace_bytes(ctypes.byref(arr[1])) > 0
    VP = ctypes.c_void_p * 2
    ptrs = VP(8, 8)
    assert L.jk_build_batched(0, arr, ptrs, ptrs, ptrs, ptrs, ptrs, 256, need, None) == _lib.JK_EINVAL
    mixed = (_lib.Problem * 2)(_prob(), _prob(precision=1))
    assert L.jk_build_batched(2, mixed, ptrs, ptrs, ptrs, ptrs, ptrs, 256, need, None) == _lib.JK_EINVAL
    nulls = VP(8, None)
    assert L.jk_build_batched(2, arr, ptrs, nulls, ptrs, ptrs, ptrs, 256, need, None) == _lib.JK_EINVAL
    assert L.jk_build_batched(2, arr, ptrs, ptrs, ptrs, ptrs, ptrs, 256, need - 1, None) == _lib.JK_EWORKSPACE


def test_status_strings():
    for s in range(6):
        assert len(_lib.status_str(s)) > 0
        assert "unknown" not in _lib.status_str(s)
    assert "unknown" in _lib.status_str(99)


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_2608_06536_amd import jk
    B = torch.zeros((2, 4, 4), dtype=torch.float64)
    C = torch.zeros((1, 4, 2), dtype=torch.float64)
    with pytest.raises(ValueError):
        jk.jk_build(B, C, C)


@pytest.mark.parametrize("ns", [1, 2, 3, 5])
def test_mixed_digit_count_unsupported(ns):
    # Only 4 digits per operand are implemented: any other count is rejected
    # by host logic before any HIP call (the pointers are never touched).
    L = _lib.lib()
    p = _prob(precision=1, nslice=ns)
    need = L.jk_workspace_bytes(ctypes.byref(p))
    assert need > 0
    assert L.jk_build(ctypes.byref(p), 8, 8, 8, 8, 8, 256, need, None) == _lib.JK_EUNSUPPORTED


def test_fock_validation():
    L = _lib.lib()
    p = _prob()
    need = L.jk_fock_workspace_bytes(ctypes.byref(p), 0)
    assert need > 0 and need % 256 == 0
    assert L.jk_fock_workspace_bytes(ctypes.byref(p), 7) == need
    assert L.jk_fock_workspace_bytes(ctypes.byref(p), -1) == 0
    assert L.jk_fock_workspace_bytes(ctypes.byref(_prob(nao=0)), 0) == 0
    c = (ctypes.c_double * 3)(2.0, -1.0, 0.0)
    clr = (ctypes.c_double * 3)(2.0, -1.0, -0.5)
    cnan = (ctypes.c_double * 3)(2.0, float("nan"), 0.0)
    F = L.jk_fock
    # B_lr and naux_lr must agree; c_lr needs B_lr
    assert F(ctypes.byref(p), 8, None, 5, 8, 8, c, 8, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, 8, 0, 8, 8, c, 8, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, clr, 8, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, cnan, 8, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, None, 8, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, c, None, 256, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, c, 8, 264, need, None) == _lib.JK_EINVAL
    assert F(ctypes.byref(p), 8, None, 0, 8, 8, c, 8, 256, need - 1, None) == _lib.JK_EWORKSPACE
    assert F(ctypes.byref(_prob(flags=1)), 8, None, 0, 8, 8, c, 8, 256, need,
             None) == _lib.JK_EINVAL


def test_vjp_block_beyond_buffer_reach_unsupported():
    # one slab's [P' | R'] block of nao x 2R doubles must stay below 4 GiB
    # (stages C and D read it through one buffer resource): the derivative
    # refuses such a problem before any launch
    L = _lib.lib()
    p = _prob(nao=16384, naux=1, ndens=1, rank=16384)       # 16384 * 2 * 16384 * 8 B = 4 GiB
    need = L.jk_workspace_bytes(ctypes.byref(p))
    assert need > 0
    assert L.jk_vjp(ctypes.byref(p), 8, 8, 8, 8, 8, 8, 8, 8, 256, need, None) == _lib.JK_EUNSUPPORTED


def test_packed_b_paths_validate():
    # packed slabs are valid for every entry point; each still refuses a
    # workspace one byte short before any launch
    L = _lib.lib()
    p = _prob(flags=_lib.JK_B_PACKED)
    need = L.jk_workspace_bytes(ctypes.byref(p))
    assert need > 0
    assert L.jk_vjp(ctypes.byref(p), 8, 8, 8, 8, 8, 8, 8, 8, 256, need - 1, None) == _lib.JK_EWORKSPACE
    for prec in (0, 1):
        arr = (_lib.Problem * 2)(_prob(flags=_lib.JK_B_PACKED, precision=prec),
                                 _prob(nao=20, flags=_lib.JK_B_PACKED, precision=prec))
        nb = L.jk_batched_workspace_bytes(2, arr)
        assert nb > 0
        VP = ctypes.c_void_p * 2
        ptrs = VP(8, 8)
        assert L.jk_build_batched(2, arr, ptrs, ptrs, ptrs, ptrs, ptrs, 256, nb - 1,
                                  None) == _lib.JK_EWORKSPACE
    # flags: both-or-neither of J and K for jk_fock, packed allowed
    c = (ctypes.c_double * 3)(2.0, -1.0, 0.0)
    pj = _prob(flags=_lib.JK_WANT_J | _lib.JK_B_PACKED)
    assert L.jk_fock(ctypes.byref(pj), 8, None, 0, 8, 8, c, 8, 256, need, None) == _lib.JK_EINVAL


def test_tuning_table_json_round_trip():
    from paper_2608_06536_amd import jk
    L = _lib.lib()
    jk.tuning_clear()
    p1 = _prob(nao=300, ndens=4, rank=30)
    p2 = _prob(nao=100, ndens=6, rank=10, precision=1)
    assert jk.tuning_get(p1) == {"ht_tile": 4, "chunk_mb": 1024}        # default
    assert jk.tuning_get(_prob(nao=500, ndens=8, rank=40))["ht_tile"] == 4
    jk.tuning_set(p1, 1, 256)
    jk.tuning_set(p2, 0, 128)
    # same shape class (nao and R in steps of 64): same entry
    assert jk.tuning_get(_prob(nao=290, ndens=2, rank=60)) == {"ht_tile": 1, "chunk_mb": 256}
    text = jk.tuning_save()
    jk.tuning_clear()
    assert jk.tuning_get(p1)["chunk_mb"] == 1024
    jk.tuning_load(text)
    assert jk.tuning_get(p1) == {"ht_tile": 1, "chunk_mb": 256}
    assert jk.tuning_get(p2) == {"ht_tile": 0, "chunk_mb": 128}
    assert jk.tuning_save() == text
    # a truncated buffer still reports the size it needs
    n = L.jk_tuning_save(None, 0)
    buf = ctypes.create_string_buffer(8)
    assert L.jk_tuning_save(buf, 8) == n and len(buf.value) == 7
    jk.tuning_clear()


@pytest.mark.parametrize("bad", [
    "", "{}", "[]", '{"version": 2, "entries": []}', '{"entries": [{"nao64": 1}]}',
    '{"version": 1, "entries": [{"nao64": 1, "rank64": 1, "precision": 0, "packed": 0, '
    '"ht_tile": 5, "chunk_mb": 256}]}',
    '{"version": 1, "entries": [{"nao64": 1, "rank64": 1, "precision": 0, "packed": 0, '
    '"ht_tile": 0, "chunk_mb": 32}]}',
    '{"version": 1, "entries": [{"nao64": 1, "rank64": 1, "precision": 0, "packed": 0, '
    '"ht_tile": 0, "chunk_mb": 256, "x": 1}]}',
    '{"version": 1, "entries": [{"nao64": 1, "rank64": 1, "precision": 0, "packed": 0, '
    '"ht_tile": 0, "chunk_mb": 256}] trailing',
])
def test_tuning_load_rejects(bad):
    L = _lib.lib()
    L.jk_tuning_clear()
    assert L.jk_tuning_load(bad.encode()) == _lib.JK_EINVAL
    n = L.jk_tuning_save(None, 0)
    buf = ctypes.create_string_buffer(n)
    L.jk_tuning_save(buf, n)
    assert b"nao64" not in buf.value          # nothing recorded


def test_tuning_validation():
    L = _lib.lib()
    p = _prob()
    for t in [(5, 256), (0, 63), (0, 4097), (-1, 256)]:
        tt = _lib.Tuning(*t)
        assert L.jk_tuning_set(ctypes.byref(p), ctypes.byref(tt)) == _lib.JK_EINVAL
    tt = _lib.Tuning(0, 256)
    assert L.jk_tuning_set(ctypes.byref(_prob(nao=0)), ctypes.byref(tt)) == _lib.JK_EINVAL
    assert L.jk_tuning_get(ctypes.byref(_prob(nao=0)), ctypes.byref(tt)) == _lib.JK_EINVAL
    need = L.jk_workspace_bytes(ctypes.byref(p))
    assert L.jk_autotune(ctypes.byref(p), 8, 8, 8, 8, 8, 256, need, None, -1,
                         None) == _lib.JK_EINVAL
    assert L.jk_autotune(ctypes.byref(p), 8, 8, 8, 8, 8, 256, need - 1, None, 2,
                         None) == _lib.JK_EWORKSPACE
    assert L.jk_autotune(ctypes.byref(p), None, 8, 8, 8, 8, 256, need, None, 2,
                         None) == _lib.JK_EINVAL
    L.jk_tuning_clear()


def test_slices_validation():
    # prepared digit planes of B (jk_slice_b / jk_build_sliced): JK_MIXED only,
    # sizes and pointers checked before any launch
    L = _lib.lib()
    p64 = _prob()
    pm = _prob(precision=1)
    assert L.jk_slices_bytes(ctypes.byref(p64)) == 0
    n = L.jk_slices_bytes(ctypes.byref(pm))
    assert n > 0 and n % 256 == 0
    # the planes depend on nao and naux only
    assert L.jk_slices_bytes(ctypes.byref(_prob(precision=1, ndens=5, rank=7))) == n
    assert L.jk_slice_b(ctypes.byref(p64), 8, 256, n, None) == _lib.JK_EINVAL
    assert L.jk_slice_b(ctypes.byref(pm), 8, None, n, None) == _lib.JK_EINVAL
    assert L.jk_slice_b(ctypes.byref(pm), 8, 264, n, None) == _lib.JK_EINVAL       # misaligned
    assert L.jk_slice_b(ctypes.byref(pm), 8, 256, n - 1, None) == _lib.JK_EWORKSPACE
    assert L.jk_slice_b(ctypes.byref(_prob(precision=1, nslice=5)), 8, 256, n,
                        None) == _lib.JK_EUNSUPPORTED
    need = L.jk_workspace_bytes(ctypes.byref(pm))
    assert L.jk_build_sliced(ctypes.byref(p64), 8, 256, n, 8, 8, 8, 8, 256, need,
                             None) == _lib.JK_EINVAL
    assert L.jk_build_sliced(ctypes.byref(pm), 8, 256, n - 1, 8, 8, 8, 8, 256, need,
                             None) == _lib.JK_EWORKSPACE
    assert L.jk_build_sliced(ctypes.byref(pm), 8, 256, n, 8, 8, 8, 8, 256, need - 1,
                             None) == _lib.JK_EWORKSPACE
    assert L.jk_build_sliced(ctypes.byref(pm), 8, None, n, 8, 8, 8, 8, 256, need,
                             None) == _lib.JK_EINVAL
