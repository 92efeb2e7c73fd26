"""GPU parity of the batched build (jk_build_batched): many problems of uneven
size per call.  Each member must be within 1e-12 of the oracle and, for
members whose slabs fit one chunk in both the batched and the single plan (all
members here), bit-identical to a single jk_build (same summation order).
On a non-default stream the launch sequence is captured into a graph on the
first call and replayed afterwards; every replay is checked, with eager work
and new data between replays."""
import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _problems(nao_list, seed=77, naux_mult=2):
    out = []
    for g, nao in enumerate(nao_list):
        naux = max(1, naux_mult * nao)
        p = synth.Problem(nao=nao, naux=naux, nd=3, r=max(1, nao // 10), ell=10.0,
                          tau=naux / 4.0 + 1, n_ground=1, seed=seed * 100 + g)
        out.append(p)
    return out


def _make(probs, scale=1.0):
    items, host = [], []
    for p in probs:
        B, CL, CR = synth.make_problem(p)
        B = B * scale
        host.append((B, CL, CR))
        items.append(tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (B, CL, CR)))
    return items, host


NAO = [23, 64, 130, 7, 100, 50, 1, 129]


def test_batched_equals_single_and_oracle():
    from paper_2608_06536_amd import jk
    probs = _problems(NAO)
    items, host = _make(probs)
    res = jk.jk_build_batched(items)
    torch.cuda.synchronize()
    for (Bd, Ld, Rd), (J, K), (B, CL, CR) in zip(items, res, host):
        Js, Ks = jk.jk_build(Bd, Ld, Rd)
        torch.cuda.synchronize()
        assert torch.equal(J, Js) and torch.equal(K, Ks)
        Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
        assert rel_err(J.cpu().numpy(), Jr) <= TOL
        assert rel_err(K.cpu().numpy(), Kr) <= TOL


def test_batched_flags():
    from paper_2608_06536_amd import jk
    probs = _problems([40, 90, 17])
    items, _ = _make(probs)
    full = jk.jk_build_batched(items)
    only_j = jk.jk_build_batched(items, want_k=False)
    only_k = jk.jk_build_batched(items, want_j=False)
    torch.cuda.synchronize()
    for (J, K), (Jo, Ko), (Jk, Kk) in zip(full, only_j, only_k):
        assert Ko is None and Jk is None
        assert torch.equal(J, Jo) and torch.equal(K, Kk)


def test_batched_graph_replays():
    # Non-default stream: first call captures, later calls replay.  Between
    # replays: eager single builds on the same stream and new input values.
    from paper_2608_06536_amd import jk
    probs = _problems([31, 77, 140, 5, 64])
    stream = torch.cuda.Stream()
    nbytes = jk.batched_workspace_bytes([jk.make_problem(p.nao, p.naux, p.nd, p.r) for p in probs])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for rep in range(4):
        items, _ = _make(probs, scale=1.0 + 0.25 * rep)
        outs = [(torch.empty((p.nd, p.nao, p.nao), dtype=torch.float64, device="cuda"),
                 torch.empty((p.nd, p.nao, p.nao), dtype=torch.float64, device="cuda")) for p in probs]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            res = jk.jk_build_batched(items, outs=outs, ws=ws)
            singles = [jk.jk_build(*it) for it in items]   # eager work on the same stream
        stream.synchronize()
        for (J, K), (Js, Ks) in zip(res, singles):
            assert torch.equal(J, Js), rep
            assert torch.equal(K, Ks), rep


def test_batched_mixed():
    from paper_2608_06536_amd import jk
    probs = _problems([45, 120, 9])
    items, host = _make(probs)
    res = jk.jk_build_batched(items, precision="mixed")
    torch.cuda.synchronize()
    for (J, K), (B, CL, CR) in zip(res, host):
        Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
        assert rel_err(J.cpu().numpy(), Jr) <= TOL
        for k in range(K.shape[0]):
            assert rel_err(K[k].cpu().numpy(), Kr[k]) <= 1e-8


def test_batched_member_over_several_chunks():
    # nao = 300, naux = 1200, 6 densities of rank 30.  Under a 256 MiB plan
    # the member runs as 4 chunks in the batch and is bit-identical to a single
    # build under that plan; under the default 1 GiB plan it is one chunk and
    # bit-identical to the default single build.  Both agree to rounding.
    from paper_2608_06536_amd import jk
    probs = [synth.Problem(nao=300, naux=1200, nd=6, r=30, ell=20.0, tau=300.0, n_ground=1,
                           seed=8801),
             synth.Problem(nao=90, naux=360, nd=6, r=9, ell=20.0, tau=90.0, n_ground=1, seed=8802)]
    items, host = _make(probs)
    p0 = probs[0]
    prob = jk.make_problem(p0.nao, p0.naux, p0.nd, p0.r)
    try:
        jk.tuning_set(prob, 4, 256)
        assert jk.plan_describe(prob)["chunk_slabs"] < p0.naux
        res_c = jk.jk_build_batched(items)
        Js, Ks = jk.jk_build(*items[0])
    finally:
        jk.tuning_clear()
    assert jk.plan_describe(prob)["chunk_slabs"] == p0.naux
    res = jk.jk_build_batched(items)
    Jd, Kd = jk.jk_build(*items[0])
    torch.cuda.synchronize()
    assert torch.equal(res_c[0][0], Js) and torch.equal(res_c[0][1], Ks)
    assert torch.equal(res[0][0], Jd) and torch.equal(res[0][1], Kd)
    assert torch.equal(res_c[0][0], res[0][0])
    assert rel_err(res_c[0][1].cpu().numpy(), res[0][1].cpu().numpy()) <= TOL
    B, CL, CR = host[0]
    Jr, Kr, _ = oracle.jk_factored(B, CL, CR)
    for J, K in (res_c[0], res[0]):
        assert rel_err(J.cpu().numpy(), Jr) <= TOL
        assert rel_err(K.cpu().numpy(), Kr) <= TOL


def test_batched_graph_cache_eviction():
    # 34 shape signatures on one non-default stream, more than the 32 graphs
    # the library keeps: the oldest are destroyed on the way (after a device
    # synchronisation).  Every call, and a later replay of the first shape
    # (captured anew), matches the single builds.
    from paper_2608_06536_amd import jk
    stream = torch.cuda.Stream()
    shapes = [[5 + g, 3 + (g % 7)] for g in range(34)] + [[5, 3]]
    for g, naos in enumerate(shapes):
        probs = _problems(naos, seed=300 + g % 34)
        items, _ = _make(probs)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            res = jk.jk_build_batched(items)
            singles = [jk.jk_build(*it) for it in items]
        stream.synchronize()
        for (J, K), (Js, Ks) in zip(res, singles):
            assert torch.equal(J, Js) and torch.equal(K, Ks), g


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_symmetric_members_and_single_plans(precision):
    # Members whose C_L and C_R are one buffer take the X-only path (upper
    # triangle, mirrored).  Every member equals a single jk_build of it bit
    # for bit under a plan whose chunks match the batch's (1 GiB for FP64,
    # 256 MiB for mixed members), and the oracle to the path's tolerance.
    from paper_2608_06536_amd import jk
    tol = TOL if precision == "fp64" else 1e-8
    chunk_mb = 1024 if precision == "fp64" else 256
    probs = _problems([70, 150, 33, 260, 9], seed=91, naux_mult=3)
    items, host = _make(probs)
    sym = [True, False, True, True, False]
    items = [(B, L, L if s else R) for (B, L, R), s in zip(items, sym)]
    res = jk.jk_build_batched(items, precision=precision)
    torch.cuda.synchronize()
    try:
        for g, ((Bd, Ld, Rd), (J, K), (B, CL, CR), p, s) in enumerate(zip(items, res, host, probs, sym)):
            jk.tuning_set(jk.make_problem(p.nao, p.naux, p.nd, p.r, precision), 4, chunk_mb)
            Js, Ks = jk.jk_build(Bd, Ld, Rd, precision=precision)
            torch.cuda.synchronize()
            assert torch.equal(J, Js), g
            assert torch.equal(K, Ks), g
            CRh = CL if s else CR
            Jr, Kr, _ = oracle.jk_factored(B, CL, CRh)
            assert rel_err(J.cpu().numpy(), Jr) <= TOL
            for k in range(p.nd):
                assert rel_err(K[k].cpu().numpy(), Kr[k]) <= tol, (g, k)
            if s:
                assert torch.equal(K, K.transpose(1, 2)), g
    finally:
        jk.tuning_clear()


def test_batched_mixed_graph_replays():
    # the mixed batch on a non-default stream: captured once, replayed with
    # new inputs and eager single builds between the replays
    from paper_2608_06536_amd import jk
    probs = _problems([31, 77, 140, 5, 64], seed=33)
    stream = torch.cuda.Stream()
    nbytes = jk.batched_workspace_bytes([jk.make_problem(p.nao, p.naux, p.nd, p.r, "mixed")
                                         for p in probs])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    try:
        for p in probs:
            jk.tuning_set(jk.make_problem(p.nao, p.naux, p.nd, p.r, "mixed"), 4, 256)
        for rep in range(3):
            items, _ = _make(probs, scale=1.0 + 0.5 * rep)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                res = jk.jk_build_batched(items, precision="mixed", ws=ws)
                singles = [jk.jk_build(*it, precision="mixed") for it in items]
            stream.synchronize()
            for (J, K), (Js, Ks) in zip(res, singles):
                assert torch.equal(J, Js), rep
                assert torch.equal(K, Ks), rep
    finally:
        jk.tuning_clear()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_packed_members(precision):
    # Every member's B packed (jk.h JK_B_PACKED), general and symmetric
    # densities mixed: each member equals a single packed jk_build of it bit
    # for bit under a plan whose chunks match the batch's, and the oracle to
    # the path's tolerance.
    from paper_2608_06536_amd import jk
    tol = TOL if precision == "fp64" else 1e-8
    chunk_mb = 1024 if precision == "fp64" else 256
    probs = _problems([70, 150, 33, 260, 9], seed=95, naux_mult=3)
    items, host = _make(probs)
    sym = [False, True, False, True, True]
    packed = []
    for (Bd, Ld, Rd), s in zip(items, sym):
        iu = torch.triu_indices(Bd.shape[1], Bd.shape[1], device="cuda")
        packed.append((Bd[:, iu[0], iu[1]].contiguous(), Ld, Ld if s else Rd))
    res = jk.jk_build_batched(packed, precision=precision)
    torch.cuda.synchronize()
    try:
        for g, ((Bp, Ld, Rd), (J, K), (B, CL, CR), p, s) in enumerate(zip(packed, res, host, probs, sym)):
            jk.tuning_set(jk.make_problem(p.nao, p.naux, p.nd, p.r, precision, packed=True), 4,
                          chunk_mb)
            Js, Ks = jk.jk_build(Bp, Ld, Rd, precision=precision)
            torch.cuda.synchronize()
            assert torch.equal(J, Js), g
            assert torch.equal(K, Ks), g
            Jr, Kr, _ = oracle.jk_factored(B, CL, CL if s else CR)
            assert rel_err(J.cpu().numpy(), Jr) <= TOL
            for k in range(p.nd):
                assert rel_err(K[k].cpu().numpy(), Kr[k]) <= tol, (g, k)
    finally:
        jk.tuning_clear()


def test_batched_packed_graph_replays():
    # packed members on a non-default stream: captured once, replayed with new
    # inputs, each replay equal to the eager single builds between them
    from paper_2608_06536_amd import jk
    probs = _problems([31, 77, 140, 5], seed=37)
    stream = torch.cuda.Stream()
    nbytes = jk.batched_workspace_bytes([jk.make_problem(p.nao, p.naux, p.nd, p.r, packed=True)
                                         for p in probs])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    try:
        for p in probs:
            jk.tuning_set(jk.make_problem(p.nao, p.naux, p.nd, p.r, packed=True), 4, 1024)
        for rep in range(3):
            items, _ = _make(probs, scale=1.0 + 0.5 * rep)
            pk = []
            for Bd, Ld, Rd in items:
                iu = torch.triu_indices(Bd.shape[1], Bd.shape[1], device="cuda")
                pk.append((Bd[:, iu[0], iu[1]].contiguous(), Ld, Rd))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                res = jk.jk_build_batched(pk, ws=ws)
                singles = [jk.jk_build(*it) for it in pk]
            stream.synchronize()
            for (J, K), (Js, Ks) in zip(res, singles):
                assert torch.equal(J, Js), rep
                assert torch.equal(K, Ks), rep
    finally:
        jk.tuning_clear()
