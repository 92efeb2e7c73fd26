"""Host logic of the Python binding (no GPU): the problem descriptor that each
entry point hands to the C ABI.

The library stands in as a recorder that returns a fixed status, and the
tensor checks are relaxed to accept CPU tensors, so that only the marshalling
is exercised.  Packed slabs must reach the library as JK_B_PACKED in every
entry point: the derivative and the batched form refuse that layout
(JK_EUNSUPPORTED) before any launch, and they can only do so if they see it.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")

from paper_2608_06536_amd import _lib, jk  # noqa: E402


class _Recorder:
    """Stands in for the loaded library: records the problem of each call."""

    def __init__(self, status):
        self.status = status
        self.flags = {}

    def _rec(self, name, prob):
        self.flags[name] = ctypes.cast(prob, ctypes.POINTER(_lib.Problem)).contents.flags

    def jk_workspace_bytes(self, prob):
        return 4096

    def jk_status_str(self, status):
        return b"recorded status"

    def jk_batched_workspace_bytes(self, n, arr):
        return 4096

    def jk_vjp(self, prob, *args):
        self._rec("jk_vjp", prob)
        return self.status

    def jk_build(self, prob, *args):
        self._rec("jk_build", prob)
        return self.status

    def jk_build_batched(self, n, arr, *args):
        self._rec("jk_build_batched", arr)
        return self.status


@pytest.fixture
def recorder(monkeypatch):
    rec = _Recorder(_lib.JK_EUNSUPPORTED)
    monkeypatch.setattr(_lib, "lib", lambda: rec)
    monkeypatch.setattr(jk, "_check_tensor", lambda t, name, shape=None: None)
    monkeypatch.setattr(jk, "_stream", lambda: ctypes.c_void_p(0))
    monkeypatch.setattr(jk, "_workspace",
                        lambda nbytes, device: torch.empty(int(nbytes), dtype=torch.uint8))
    return rec


def _packed_inputs(nao=6, naux=3, nd=2, r=2):
    B = torch.zeros((naux, nao * (nao + 1) // 2), dtype=torch.float64)
    CL = torch.zeros((nd, nao, r), dtype=torch.float64)
    CR = torch.zeros((nd, nao, r), dtype=torch.float64)
    return B, CL, CR


def test_vjp_passes_packed_flag(recorder):
    B, CL, CR = _packed_inputs()
    with pytest.raises(_lib.JKError) as ei:
        jk.jk_vjp(B, CL, CR, None, None)
    assert ei.value.status == _lib.JK_EUNSUPPORTED
    assert recorder.flags["jk_vjp"] & _lib.JK_B_PACKED


def test_batched_passes_packed_flag(recorder):
    items = [_packed_inputs(), _packed_inputs(nao=9)]
    with pytest.raises(_lib.JKError) as ei:
        jk.jk_build_batched(items)
    assert ei.value.status == _lib.JK_EUNSUPPORTED
    assert recorder.flags["jk_build_batched"] & _lib.JK_B_PACKED


def test_full_slabs_carry_no_packed_flag(recorder):
    nao, naux = 6, 3
    B = torch.zeros((naux, nao, nao), dtype=torch.float64)
    _, CL, CR = _packed_inputs(nao, naux)
    with pytest.raises(_lib.JKError):
        jk.jk_vjp(B, CL, CR, None, None)
    assert not recorder.flags["jk_vjp"] & _lib.JK_B_PACKED


def test_autograd_backward_refuses_packed(recorder):
    B, CL, CR = _packed_inputs()
    recorder.status = _lib.JK_OK          # the forward build is accepted for packed B
    CL.requires_grad_(True)
    J, K = jk.jk(B, CL, CR)
    assert recorder.flags["jk_build"] & _lib.JK_B_PACKED
    recorder.status = _lib.JK_EUNSUPPORTED
    with pytest.raises(_lib.JKError) as ei:
        (J.sum() + K.sum()).backward()
    assert ei.value.status == _lib.JK_EUNSUPPORTED
    assert recorder.flags["jk_vjp"] & _lib.JK_B_PACKED
