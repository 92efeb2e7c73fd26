"""jk_build_noalloc (jk.h): the build for callers that cannot allocate device
memory.  Its kernel buffers live in the library's own device array, so the
call takes no workspace.  Checked through the C ABI against jk_build and the
oracle (FP64, normwise 1e-12) on calls in a row, each smaller than the one
before, so that a later call runs over what an earlier one left in the
shared array; then the refusal of a problem whose plan does not fit.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import _lib, jk, synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _noalloc(Bd, Ld, Rd, prob):
    nd, nao = Ld.shape[0], Ld.shape[1]
    J = torch.empty((nd, nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    st = _lib.lib().jk_build_noalloc(ctypes.byref(prob), Bd.data_ptr(), Ld.data_ptr(),
                                     Rd.data_ptr(), J.data_ptr(), K.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == _lib.JK_OK, _lib.status_str(st)
    return J, K


@pytest.mark.parametrize("order", ["large_first"])
def test_noalloc_matches_jk_build(order):
    cases = [
        synth.Problem(nao=500, naux=600, nd=8, r=40, ell=20.0, tau=150.0, n_ground=2, seed=9101),
        synth.Problem(nao=300, naux=1200, nd=4, r=30, ell=20.0, tau=300.0, n_ground=1, seed=9102),
        synth.Problem(nao=48, naux=192, nd=1, r=8, ell=8.0, tau=64.0, seed=9103),
    ]
    for i, p in enumerate(cases):
        print(f"noalloc call {i}: nao {p.nao} naux {p.naux} nd {p.nd} r {p.r}", flush=True)
        B, CL, CR = synth.make_problem(p)
        Bd, Ld, Rd = (torch.from_numpy(a).cuda() for a in (B, CL, CR))
        prob = jk.make_problem(p.nao, p.naux, p.nd, p.r)
        J, K = _noalloc(Bd, Ld, Rd, prob)
        Jr, Kr = jk.jk_build(Bd, Ld, Rd)
        torch.cuda.synchronize()
        assert torch.equal(J, Jr), i                      # J does not depend on the chunking
        assert rel_err(K.cpu().numpy(), Kr.cpu().numpy()) <= TOL, i
        Jo, Ko, _ = oracle.jk_factored(B, CL, CR)
        assert rel_err(J.cpu().numpy(), Jo) <= TOL, i
        assert rel_err(K.cpu().numpy(), Ko) <= TOL, i
        # symmetric densities: one factor buffer for both sides
        Js, Ks = _noalloc(Bd, Ld, Ld, prob)
        Jrs, Krs = jk.jk_build(Bd, Ld, Ld)
        torch.cuda.synchronize()
        assert torch.equal(Js, Jrs), i
        assert rel_err(Ks.cpu().numpy(), Krs.cpu().numpy()) <= TOL, i


def test_noalloc_refuses_oversized_and_mixed():
    L = _lib.lib()
    big = jk.make_problem(2000, 100, 16, 80)          # densities alone: 512 MB
    assert L.jk_build_noalloc(ctypes.byref(big), 8, 8, 8, 8, 8, None) == _lib.JK_EWORKSPACE
    mixed = jk.make_problem(48, 192, 1, 8, "mixed")
    assert L.jk_build_noalloc(ctypes.byref(mixed), 8, 8, 8, 8, 8, None) == _lib.JK_EUNSUPPORTED
