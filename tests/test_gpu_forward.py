"""GPU parity of the FP64 forward build (jk_build) against the CPU oracle.

Tolerance: normwise max|x - ref| / max|ref| <= 1e-12 per result (FP64 path).
Sizes span several 64-wide tiles with ragged tails; full-size inputs are
checked on entries the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrs]


def _run(B, CL, CR, **kw):
    from paper_2608_06536_amd import jk
    Bd, Ld, Rd = _dev(B, CL, CR)
    J, K = jk.jk_build(Bd, Ld, Rd, **kw)
    torch.cuda.synchronize()
    return (None if J is None else J.cpu().numpy()), (None if K is None else K.cpu().numpy())


def test_config1_vs_bruteforce():
    p = synth.config(1)
    B, CL, CR = synth.make_problem(p)
    J, K = _run(B, CL, CR)
    D = oracle.density(CL, CR)
    J0, K0 = oracle.jk_from_eri(oracle.eri4(B), D[0])
    assert rel_err(J[0], J0) <= TOL
    assert rel_err(K[0], K0) <= TOL


@pytest.mark.parametrize("nao,naux,nd,r", [
    (1, 1, 1, 1),          # degenerate
    (7, 3, 2, 3),          # smaller than one tile
    (65, 9, 3, 5),         # one past a tile edge
    (130, 37, 2, 13),      # several tiles, ragged in every dimension
    (200, 50, 5, 17),      # 2R = 170 columns: ragged column tiles
])
def test_ragged_shapes(nao, naux, nd, r):
    p = synth.Problem(nao=nao, naux=naux, nd=nd, r=r, ell=10.0, tau=naux / 4 + 1, n_ground=1,
                      seed=77 + nao)
    B, CL, CR = synth.make_problem(p)
    J, K = _run(B, CL, CR)
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    assert rel_err(J, Jr) <= TOL
    assert rel_err(K, Kr) <= TOL


def test_config2_fp64():
    p = synth.config(2)
    B, CL, CR = synth.make_problem(p)
    J, K = _run(B, CL, CR)
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    for k in range(p.nd):
        assert rel_err(J[k], Jr[k]) <= TOL, k
        assert rel_err(K[k], Kr[k]) <= TOL, k


def test_want_flags_and_determinism():
    p = synth.Problem(nao=96, naux=40, nd=2, r=6, ell=10.0, tau=20.0, seed=5)
    B, CL, CR = synth.make_problem(p)
    J1, K1 = _run(B, CL, CR)
    J2, K2 = _run(B, CL, CR)
    assert np.array_equal(J1, J2) and np.array_equal(K1, K2)   # bit-identical reruns
    Jo, Ko = _run(B, CL, CR, want_k=False)
    assert Ko is None and np.array_equal(Jo, J1)
    Jn, Kn = _run(B, CL, CR, want_j=False)
    assert Jn is None and np.array_equal(Kn, K1)


def test_invariants_on_gpu():
    # K[D^T] = K[D]^T and J[D^T] = J[D] through the library itself.
    p = synth.Problem(nao=80, naux=30, nd=2, r=5, ell=10.0, tau=30.0, seed=6)
    B, CL, CR = synth.make_problem(p)
    J, K = _run(B, CL, CR)
    Jt, Kt = _run(B, CR, CL)
    assert rel_err(Kt, K.transpose(0, 2, 1)) <= TOL
    assert rel_err(Jt, J) <= TOL


def test_config4_sampled_entries():
    # Full headline size (nao=500, naux=2000, nd=8, r=40) in the launch
    # configuration the benchmark times; entries checked one by one.
    p = synth.config(4)
    B, CL, CR = synth.make_problem(p)
    J, K = _run(B, CL, CR)
    rng = np.random.default_rng(404)
    n = 24
    ks = rng.integers(0, p.nd, n)
    ms = rng.integers(0, p.nao, n)
    ns = rng.integers(0, p.nao, n)
    ms[:4] = p.nao - 1          # ragged tail of the last tile
    ns[4:8] = p.nao - 1
    Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms, ns)
    assert np.max(np.abs(J[ks, ms, ns] - Je)) <= TOL * np.max(np.abs(J))
    assert np.max(np.abs(K[ks, ms, ns] - Ke)) <= TOL * np.max(np.abs(K))
    # properties that hold at any size
    assert rel_err(J, J.transpose(0, 2, 1)) <= TOL
    assert np.all(np.isfinite(K))
