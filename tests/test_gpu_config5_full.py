"""GPU parity at the largest workload in full: nao=1000, naux=4000 (B is
32 GB in FP64 on the device), 16 densities of rank 80, with the derivative
(dB is another 32 GB).  Entries are checked one by one against the oracle,
plus properties that hold at any size.  Inputs are generated on the host with
a thread pool (each slab has its own seeded stream).

Tolerances (normwise, max|x - ref| / max|x|): FP64 1e-12, mixed 1e-8.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_MIXED = 1e-8


def _make_B(p):
    B = np.empty((p.naux, p.nao, p.nao))
    step = 50
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda a: synth.make_B_slabs(p, range(a, min(a + step, p.naux)),
                                                 out=B[a:min(a + step, p.naux)]),
                    range(0, p.naux, step)))
    return B


def test_config5_full_forward_and_derivative():
    from paper_2608_06536_amd import jk
    p = synth.config(5)
    print(f"config 5: nao {p.nao} naux {p.naux} nd {p.nd} r {p.r}", flush=True)
    B = _make_B(p)
    CL, CR = synth.make_factors(p)
    W, V = synth.make_cotangents(p)
    dev = torch.device("cuda")
    Bd = torch.from_numpy(B).to(dev)
    Ld, Rd, Wd, Vd = (torch.from_numpy(a).to(dev) for a in (CL, CR, W, V))
    J, K = jk.jk_build(Bd, Ld, Rd)
    Jm, Km = jk.jk_build(Bd, Ld, Rd, precision="mixed")
    torch.cuda.synchronize()
    rng = np.random.default_rng(5005)
    n = 16
    ks, ms, ns = rng.integers(0, p.nd, n), rng.integers(0, p.nao, n), rng.integers(0, p.nao, n)
    ms[:3] = p.nao - 1
    ns[3:6] = p.nao - 1
    ks[6] = p.nd - 1
    Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms, ns)
    Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
    assert np.max(np.abs(Jh[ks, ms, ns] - Je)) <= TOL * np.max(np.abs(Jh))
    assert np.max(np.abs(Kh[ks, ms, ns] - Ke)) <= TOL * np.max(np.abs(Kh))
    assert torch.equal(Jm, J)
    Kmh = Km.cpu().numpy()
    for k in range(p.nd):
        assert rel_err(Kmh[k], Kh[k]) <= TOL_MIXED
    assert rel_err(Jh, Jh.transpose(0, 2, 1)) <= TOL       # J of a symmetric B is symmetric
    del Jm, Km, Kmh
    # K[D^T] = K[D]^T at full size (swap the factors)
    _, Kt = jk.jk_build(Bd, Rd, Ld, want_j=False)
    torch.cuda.synchronize()
    assert rel_err(Kt.transpose(1, 2).cpu().numpy(), Kh) <= TOL
    del Kt, J, K
    # derivative: 32 GB dB on the device
    dB, dCL, dCR = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd)
    torch.cuda.synchronize()
    qs = rng.integers(0, p.naux, 12)
    as_ = rng.integers(0, p.nao, 12)
    bs = rng.integers(0, p.nao, 12)
    qs[0] = p.naux - 1
    as_[1] = p.nao - 1
    ref = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs)
    got = dB[qs, as_, bs].cpu().numpy()
    assert np.max(np.abs(got - ref)) <= TOL * float(dB.abs().max())
    # dC_L, dC_R at full size: the one-density oracle would cost ~1e12 CPU flops
    # here; they are checked entry for entry on the 500-slab share
    # (test_gpu_large.py), and here through the self-adjoint identity
    # (Sec. 2.1, Eq. (1)): with A_k = J[W_k] + K[V_k],
    #     dC_Lk = A_k C_Rk,   dC_Rk = A_k^T C_Lk,
    # where J[W] and K[V] come from forward builds whose densities are W_k and
    # V_k themselves (left factor W_k or V_k, right factor the identity), a
    # path that shares no kernel with the derivative's stages.
    assert bool(torch.isfinite(dCL).all()) and bool(torch.isfinite(dCR).all())
    del dB
    torch.cuda.empty_cache()
    eye = torch.eye(p.nao, dtype=torch.float64, device=dev)
    for k in (0, p.nd - 1):
        F = torch.stack([Wd[k], Vd[k]])                 # densities W_k and V_k
        Jf, Kf = jk.jk_build(Bd, F, torch.stack([eye, eye]))
        A = Jf[0] + Kf[1]
        torch.cuda.synchronize()
        assert rel_err(dCL[k].cpu().numpy(), (A @ Rd[k]).cpu().numpy()) <= TOL, k
        assert rel_err(dCR[k].cpu().numpy(), (A.T.contiguous() @ Ld[k]).cpu().numpy()) <= TOL, k
        del Jf, Kf, A
