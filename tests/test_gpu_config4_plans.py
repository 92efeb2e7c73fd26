"""GPU parity of the plans the autotuner can pick at the headline size
(nao=500, naux=2000, 8 densities of rank 40; B is 4 GB), and of the mixed
path's int32 slice sums at the deepest exchange split a plan allows.

* Tile 4 (16x16x4 engine over stacked slabs) with 2048 and 4096 MB chunks:
  a 4096 MB chunk holds 1676 slabs, 3.35 GB of B behind one buffer
  resource.  J, K and dB against sampled oracle entries (FP64 1e-12,
  normwise), J identical across plans (it does not depend on chunks), K equal
  across plans to rounding, and the mixed build's K within 1e-8.
* The int32 cap: a sum over n inner indices of digit-pair products stays
  exact for n <= 32767.  Identity slabs and factors whose every entry is
  v = (127 2^24 - 128 2^16 + 127 2^8 - 128) / 2^31 give X and Y rows of
  constant magnitude whose digits are (127, -128, 127, -128): level 5 then
  adds 4 * (-16256) per index, -2,119,782,400 at depth 32600, the most
  negative sum these digits allow.  K and J have closed forms.
"""
import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_MIXED = 1e-8


@pytest.fixture(scope="module")
def config4():
    p = synth.config(4)
    print(f"config 4: nao {p.nao} naux {p.naux} nd {p.nd} r {p.r}", flush=True)
    B = synth.make_B_parallel(p)
    CL, CR = synth.make_factors(p)
    W, V = synth.make_cotangents(p)
    return p, B, CL, CR, W, V


def test_tile4_large_chunks(config4):
    from paper_2608_06536_amd import jk
    p, B, CL, CR, W, V = config4
    dev = torch.device("cuda")
    Bd = torch.from_numpy(B).to(dev)
    Ld, Rd, Wd, Vd = (torch.from_numpy(a).to(dev) for a in (CL, CR, W, V))
    prob = jk.make_problem(p.nao, p.naux, p.nd, p.r)
    mprob = jk.make_problem(p.nao, p.naux, p.nd, p.r, "mixed")
    rng = np.random.default_rng(4004)
    n = 24
    ks, ms, ns = rng.integers(0, p.nd, n), rng.integers(0, p.nao, n), rng.integers(0, p.nao, n)
    ms[:3] = p.nao - 1
    ns[3:6] = p.nao - 1
    ks[6] = p.nd - 1
    Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms, ns)
    qs, as_, bs = rng.integers(0, p.naux, 12), rng.integers(0, p.nao, 12), rng.integers(0, p.nao, 12)
    qs[0] = p.naux - 1
    as_[1] = p.nao - 1
    dBe = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs)
    res = {}
    try:
        for mb in (2048, 4096):
            jk.tuning_set(prob, 4, mb)
            jk.tuning_set(mprob, 4, mb)
            info = jk.plan_describe(prob)
            print(f"plan tile 4, {mb} MB: {info['chunk_slabs']} slabs per chunk", flush=True)
            J, K = jk.jk_build(Bd, Ld, Rd)
            Jm, Km = jk.jk_build(Bd, Ld, Rd, precision="mixed")
            dB, dCL, dCR = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd)
            torch.cuda.synchronize()
            Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
            assert np.max(np.abs(Jh[ks, ms, ns] - Je)) <= TOL * np.max(np.abs(Jh)), mb
            assert np.max(np.abs(Kh[ks, ms, ns] - Ke)) <= TOL * np.max(np.abs(Kh)), mb
            got = dB[qs, as_, bs].cpu().numpy()
            assert np.max(np.abs(got - dBe)) <= TOL * float(dB.abs().max()), mb
            assert bool(torch.isfinite(dCL).all()) and bool(torch.isfinite(dCR).all())
            assert torch.equal(Jm, J), mb
            Kmh = Km.cpu().numpy()
            for k in range(p.nd):
                err = np.max(np.abs(Kmh[k] - Kh[k])) / np.max(np.abs(Kh[k]))
                assert err <= TOL_MIXED, (mb, k, err)
            res[mb] = (Jh, Kh)
            del J, K, Jm, Km, dB, dCL, dCR
    finally:
        jk.tuning_clear()
    assert np.array_equal(res[2048][0], res[4096][0])
    Ka, Kb = res[2048][1], res[4096][1]
    assert np.max(np.abs(Ka - Kb)) <= TOL * np.max(np.abs(Ka))


def _digit_edge_value():
    n = 127 * 2 ** 24 - 128 * 2 ** 16 + 127 * 2 ** 8 - 128
    return n / 2.0 ** 31


@pytest.mark.parametrize("sym", [False, True])
def test_mixed_int32_sums_at_the_cap(sym):
    from paper_2608_06536_amd import jk
    # one split per chunk needs a full round of exchange tiles: nao = 2048
    # (16 x 16 tiles of 128); naux * r = 163 * 200 = 32600 inner indices
    nao, naux, nd, r = 2048, 163, 1, 200
    v = _digit_edge_value()
    assert 0.98 < v * 128 / 127 < 1.0           # row exponent 0, leading digit 127
    prob = jk.make_problem(nao, naux, nd, r, "mixed")
    try:
        jk.tuning_set(prob, 4, 4096)
        info = jk.plan_describe(prob)
        print(f"near-cap plan: {info}", flush=True)
        assert info["chunk_slabs"] == naux
        assert 32000 <= info["int_depth"] <= info["int_depth_cap"]
        if not sym:
            assert info["nsplit"] == 1
        dev = torch.device("cuda")
        Bd = torch.eye(nao, dtype=torch.float64, device=dev).expand(naux, nao, nao).contiguous()
        Ld = torch.full((nd, nao, r), v, dtype=torch.float64, device=dev)
        Rd = Ld if sym else Ld.clone()
        J, K = jk.jk_build(Bd, Ld, Rd, precision="mixed")
        torch.cuda.synchronize()
    finally:
        jk.tuning_clear()
    kref = naux * r * v * v                     # K = sum_Q C_L C_R^T, every entry
    jref = naux * (nao * r * v * v)             # J = sum_Q tr(D) I
    Kh = K.cpu().numpy()
    assert np.max(np.abs(Kh - kref)) <= TOL_MIXED * kref
    Jh = J.cpu().numpy()
    assert np.max(np.abs(np.diagonal(Jh, axis1=1, axis2=2) - jref)) <= TOL * jref
    assert np.max(np.abs(Jh - Jh * np.eye(nao))) == 0.0
