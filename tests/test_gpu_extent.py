"""GPU parity where a chunk of slabs spans 4 GiB or more (nao=1500, 300 slabs
of B in one chunk: 5.4 GB).  The stacked-slab half-transform reads the chunk
through one buffer resource, whose byte offsets stop at 4 GiB, so the build
and the derivative fall back to the 4x4x4 tile there; a 64 MB chunk keeps the
16x16x4 tile.  Both plans are checked against sampled oracle entries and
against each other.

Tolerances (normwise): FP64 1e-12.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _make_B(p):
    B = np.empty((p.naux, p.nao, p.nao))
    step = 20
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda a: synth.make_B_slabs(p, range(a, min(a + step, p.naux)),
                                                 out=B[a:min(a + step, p.naux)]),
                    range(0, p.naux, step)))
    return B


def test_chunk_beyond_buffer_reach():
    from paper_2608_06536_amd import jk
    p = synth.Problem(nao=1500, naux=300, nd=2, r=16, ell=30.0, tau=120.0, seed=7300)
    print(f"nao {p.nao} naux {p.naux}: B {p.naux * p.nao ** 2 * 8 / 2 ** 30:.1f} GiB", flush=True)
    B = _make_B(p)
    CL, CR = synth.make_factors(p)
    W, V = synth.make_cotangents(p)
    dev = torch.device("cuda")
    Bd = torch.from_numpy(B).to(dev)
    Ld, Rd, Wd, Vd = (torch.from_numpy(a).to(dev) for a in (CL, CR, W, V))
    prob = jk.make_problem(p.nao, p.naux, p.nd, p.r)
    out = {}
    for mb in (64, 1024):           # 87 slabs (1.6 GB) per chunk, or all 300 (5.4 GB)
        jk.tuning_set(prob, 4, mb)
        J, K = jk.jk_build(Bd, Ld, Rd)
        torch.cuda.synchronize()
        out[mb] = (J.cpu().numpy(), K.cpu().numpy())
    jk.tuning_clear()
    rng = np.random.default_rng(7301)
    n = 24
    ks, ms, ns = rng.integers(0, p.nd, n), rng.integers(0, p.nao, n), rng.integers(0, p.nao, n)
    ms[:3] = p.nao - 1
    ns[3:6] = p.nao - 1
    Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms, ns)
    for mb, (Jh, Kh) in out.items():
        assert np.max(np.abs(Jh[ks, ms, ns] - Je)) <= TOL * np.max(np.abs(Jh)), mb
        assert np.max(np.abs(Kh[ks, ms, ns] - Ke)) <= TOL * np.max(np.abs(Kh)), mb
    Ka, Kb = out[64][1], out[1024][1]
    assert np.max(np.abs(Ka - Kb)) <= TOL * np.max(np.abs(Ka))
    assert np.array_equal(out[64][0], out[1024][0])            # J does not depend on chunks
    del out
    # the derivative: its 4 GiB chunks hold all 300 slabs, too
    dB, dCL, dCR = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd)
    torch.cuda.synchronize()
    qs, as_, bs = rng.integers(0, p.naux, 12), rng.integers(0, p.nao, 12), rng.integers(0, p.nao, 12)
    qs[0] = p.naux - 1
    as_[1] = p.nao - 1
    ref = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs)
    got = dB[qs, as_, bs].cpu().numpy()
    assert np.max(np.abs(got - ref)) <= TOL * float(dB.abs().max())
    assert bool(torch.isfinite(dCL).all()) and bool(torch.isfinite(dCR).all())
