"""GPU parity of the symmetric-density case: the same factor passed for both
sides (C_L = C_R, so every D_k = C_k C_k^T is symmetric).  The build then
forms only X = B^Q C and K = sum X X^T on the upper-triangle tiles, mirrored.

Checked against the oracle with C_R = C_L (FP64 1e-12, mixed 1e-8), against
the general path on a copy of the factor, and K must be exactly symmetric.
"""
import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_MIXED = 1e-8


def _problem(nao, naux, nd, r, seed):
    p = synth.Problem(nao=nao, naux=naux, nd=nd, r=r, ell=10.0, tau=naux / 4.0 + 1, n_ground=nd,
                      seed=seed)
    B, CL, _ = synth.make_problem(p)
    return B, CL


@pytest.mark.parametrize("nao,naux,nd,r", [(1, 1, 1, 1), (23, 17, 2, 5), (130, 37, 3, 13),
                                           (200, 50, 5, 17), (257, 20, 1, 64)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_symmetric_vs_oracle(nao, naux, nd, r, precision):
    from paper_2608_06536_amd import jk
    B, C = _problem(nao, naux, nd, r, seed=7000 + nao)
    Bd = torch.from_numpy(B).cuda()
    Cd = torch.from_numpy(C).cuda()
    J, K = jk.jk_build(Bd, Cd, Cd, precision=precision)          # same tensor: symmetric path
    Jg, Kg = jk.jk_build(Bd, Cd, Cd.clone(), precision=precision)  # general path
    torch.cuda.synchronize()
    Jr, Kr, _ = oracle.jk_factored(B, C, C)
    Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
    tol = TOL if precision == "fp64" else TOL_MIXED
    assert rel_err(Jh, Jr) <= TOL
    for k in range(nd):
        assert rel_err(Kh[k], Kr[k]) <= tol
        assert rel_err(Kh[k], Kg[k].cpu().numpy()) <= 2 * tol
    assert np.array_equal(Kh, Kh.transpose(0, 2, 1))
    assert torch.equal(J, Jg)


def test_symmetric_config4_sampled():
    # headline size with ground-state-like densities (C_L = C_R)
    from paper_2608_06536_amd import jk
    p = synth.config(4)
    B = synth.make_B(p)
    C, _ = synth.make_factors(p)
    Bd, Cd = torch.from_numpy(B).cuda(), torch.from_numpy(C).cuda()
    J, K = jk.jk_build(Bd, Cd, Cd)
    Jm, Km = jk.jk_build(Bd, Cd, Cd, precision="mixed")
    torch.cuda.synchronize()
    rng = np.random.default_rng(4004)
    n = 24
    ks, ms, ns = rng.integers(0, p.nd, n), rng.integers(0, p.nao, n), rng.integers(0, p.nao, n)
    ms[:4] = p.nao - 1
    ns[4:8] = p.nao - 1
    Je, Ke = oracle.jk_entries(B, C, C, ks, ms, ns)
    Jh, Kh, Kmh = J.cpu().numpy(), K.cpu().numpy(), Km.cpu().numpy()
    assert np.max(np.abs(Jh[ks, ms, ns] - Je)) <= TOL * np.max(np.abs(Jh))
    assert np.max(np.abs(Kh[ks, ms, ns] - Ke)) <= TOL * np.max(np.abs(Kh))
    assert np.array_equal(Kh, Kh.transpose(0, 2, 1))
    for k in range(p.nd):
        assert rel_err(Kmh[k], Kh[k]) <= TOL_MIXED
