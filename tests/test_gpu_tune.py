"""GPU checks of plan autotuning (jk_tune.h): every plan computes the same J
and K (oracle 1e-12 FP64, 1e-8 mixed); a tile choice alone is bit-identical
to the default plan; jk_autotune records a plan that later builds reuse
(bit-identical reruns); batched members follow their class's chunk budget.
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


@pytest.fixture(autouse=True)
def clean_table():
    from paper_2608_06536_amd import jk
    jk.tuning_clear()
    yield
    jk.tuning_clear()


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrs]


def _case(nao, naux, nd, r, seed):
    p = synth.Problem(nao=nao, naux=naux, nd=nd, r=r, ell=10.0, tau=naux / 4.0 + 1, seed=seed)
    return synth.make_problem(p)


@pytest.mark.parametrize("nao,naux,nd,r", [(130, 37, 3, 13), (300, 120, 4, 30), (65, 9, 2, 64)])
def test_tile_choice_is_bit_identical(nao, naux, nd, r):
    from paper_2608_06536_amd import jk
    B, CL, CR = _case(nao, naux, nd, r, 7100 + nao)
    Bd, Ld, Rd = _dev(B, CL, CR)
    prob = jk.make_problem(nao, naux, nd, r)
    jk.tuning_set(prob, 0, 1024)
    J0, K0 = jk.jk_build(Bd, Ld, Rd)
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    for tile in (1, 2, 3, 4):
        jk.tuning_set(prob, tile, 1024)
        J1, K1 = jk.jk_build(Bd, Ld, Rd)
        torch.cuda.synchronize()
        assert torch.equal(J0, J1) and torch.equal(K0, K1)
        for k in range(nd):
            assert rel_err(K1[k].cpu().numpy(), Kr[k]) <= TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mb", [64, 128])
def test_chunk_choice_vs_oracle(precision, mb):
    from paper_2608_06536_amd import jk
    p = synth.config(2)                        # nao 300, naux 1200, 4 densities of rank 30
    B, CL, CR = synth.make_problem(p)
    Bd, Ld, Rd = _dev(B, CL, CR)
    jk.tuning_set(jk.make_problem(p.nao, p.naux, p.nd, p.r, precision), 0, mb)
    J, K = jk.jk_build(Bd, Ld, Rd, precision=precision)
    torch.cuda.synchronize()
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    tol = TOL if precision == "fp64" else TOL_MIXED
    for k in range(p.nd):
        assert rel_err(J[k].cpu().numpy(), Jr[k]) <= TOL
        assert rel_err(K[k].cpu().numpy(), Kr[k]) <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_records_and_reproduces(precision):
    from paper_2608_06536_amd import jk
    B, CL, CR = _case(200, 300, 3, 20, 7200)
    Bd, Ld, Rd = _dev(B, CL, CR)
    J, K, choice = jk.autotune(Bd, Ld, Rd, precision=precision)
    prob = jk.make_problem(200, 300, 3, 20, precision)
    assert jk.tuning_get(prob) == choice
    assert choice["chunk_mb"] in (128, 256, 512, 1024, 2048, 4096)
    assert choice["ht_tile"] in ((2, 3, 4) if precision == "fp64" else (4,))
    J2, K2 = jk.jk_build(Bd, Ld, Rd, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(J, J2) and torch.equal(K, K2)
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    tol = TOL if precision == "fp64" else TOL_MIXED
    for k in range(3):
        assert rel_err(J[k].cpu().numpy(), Jr[k]) <= TOL
        assert rel_err(K[k].cpu().numpy(), Kr[k]) <= tol


@pytest.mark.parametrize("tiles", [(0, 0, 0), (1, 0, 1), (1, 1, 1), (2, 1, 2), (4, 3, 1)])
def test_batched_follows_class_plans(tiles):
    # members of one batch with different half-transform tiles and chunk budgets
    from paper_2608_06536_amd import jk
    probs = synth.batched_problems(nao_list=[100, 130, 257])
    items, host, singles = [], [], []
    for q, t in zip(probs, tiles):
        B, CL, CR = synth.make_problem(q)
        host.append((B, CL, CR))
        items.append(tuple(_dev(B, CL, CR)))
        jk.tuning_set(jk.make_problem(q.nao, q.naux, q.nd, q.r), t, 64 if t else 128)
    res = jk.jk_build_batched(items)
    for Bd, Ld, Rd in items:
        singles.append(jk.jk_build(Bd, Ld, Rd))
    torch.cuda.synchronize()
    for (B, CL, CR), (J, K), (Js, Ks) in zip(host, res, singles):
        assert torch.equal(J, Js) and torch.equal(K, Ks)      # a member computes as alone
        Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
        for k in range(CL.shape[0]):
            assert rel_err(J[k].cpu().numpy(), Jr[k]) <= TOL
            assert rel_err(K[k].cpu().numpy(), Kr[k]) <= TOL


def test_autotune_batched_classes():
    from paper_2608_06536_amd import jk
    probs = synth.batched_problems(nao_list=[100, 105, 300])
    items = [tuple(_dev(*synth.make_problem(q))) for q in probs]
    plans = jk.autotune_batched(items)
    assert len(plans) == 2                       # nao 100 and 105 (rank 10) share a class
    for q in probs:
        got = jk.tuning_get(jk.make_problem(q.nao, q.naux, q.nd, q.r))
        assert got in plans.values()
    res = jk.jk_build_batched(items)
    torch.cuda.synchronize()
    for q, (J, K) in zip(probs, res):
        B, CL, CR = synth.make_problem(q)
        Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
        for k in range(q.nd):
            assert rel_err(K[k].cpu().numpy(), Kr[k]) <= TOL


def test_q_blocking_independence():
    # The Q-chunk is a memory knob: 64 MB and 1 GB chunks (different launch
    # counts and exchange splits) agree to rounding, and each is bit-identical
    # on a rerun.
    from paper_2608_06536_amd import jk
    p = synth.config(2)
    B, CL, CR = synth.make_problem(p)
    Bd, Ld, Rd = _dev(B, CL, CR)
    prob = jk.make_problem(p.nao, p.naux, p.nd, p.r)
    out = {}
    for mb in (64, 1024):
        jk.tuning_set(prob, 0, mb)
        a = jk.jk_build(Bd, Ld, Rd)
        b = jk.jk_build(Bd, Ld, Rd)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        out[mb] = a
    for t in (0, 1):
        for k in range(p.nd):
            assert rel_err(out[64][t][k].cpu().numpy(), out[1024][t][k].cpu().numpy()) <= 1e-14
