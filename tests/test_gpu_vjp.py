"""GPU parity of the reverse-mode derivative (jk_vjp) against the CPU oracle,
central differences through the GPU forward, the self-adjoint identity and
torch.autograd.  FP64 tolerance: normwise 1e-12 per result."""
import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dev(*arrs):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrs]


def _np(t):
    return None if t is None else t.cpu().numpy()


def _vjp(B, CL, CR, W, V, **kw):
    from paper_2608_06536_amd import jk
    Bd, Ld, Rd, Wd, Vd = _dev(B, CL, CR, W, V)
    out = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd, **kw)
    torch.cuda.synchronize()
    return [_np(t) for t in out]


def _prob(nao, naux, nd, r, seed):
    p = synth.Problem(nao=nao, naux=naux, nd=nd, r=r, ell=10.0, tau=naux / 4 + 1, n_ground=1,
                      seed=seed)
    B, CL, CR = synth.make_problem(p)
    W, V = synth.make_cotangents(p)
    return B, CL, CR, W, V


@pytest.mark.parametrize("nao,naux,nd,r", [
    (1, 1, 1, 1),
    (9, 4, 2, 3),
    (70, 11, 3, 7),
    (131, 21, 2, 20),     # 3R = 120: inner dimension not a multiple of 16
    (48, 192, 1, 8),      # the nao=48 workload shape
    (50, 30, 8, 5),       # omega and gamma as 16 projections in one pass over B
    (45, 20, 5, 4),       # 10 of the 16 projection columns used
    (40, 15, 9, 3),       # 18 projections: omega and gamma in passes of their own
])
def test_vjp_vs_oracle(nao, naux, nd, r):
    B, CL, CR, W, V = _prob(nao, naux, nd, r, 300 + nao)
    dB, dCL, dCR = _vjp(B, CL, CR, W, V)
    rB, rL, rR = oracle.vjp(B, CL, CR, W, V)
    assert rel_err(dB, rB) <= TOL
    assert rel_err(dCL, rL) <= TOL
    assert rel_err(dCR, rR) <= TOL


@pytest.mark.parametrize("which", ["W", "V"])
def test_vjp_single_cotangent(which):
    B, CL, CR, W, V = _prob(60, 13, 2, 5, 11)
    W = W if which == "W" else None
    V = V if which == "V" else None
    dB, dCL, dCR = _vjp(B, CL, CR, W, V)
    rB, rL, rR = oracle.vjp(B, CL, CR, W, V)
    assert rel_err(dB, rB) <= TOL and rel_err(dCL, rL) <= TOL and rel_err(dCR, rR) <= TOL


def test_vjp_partial_outputs_and_determinism():
    B, CL, CR, W, V = _prob(77, 17, 2, 6, 12)
    full = _vjp(B, CL, CR, W, V)
    again = _vjp(B, CL, CR, W, V)
    for a, b in zip(full, again):
        assert np.array_equal(a, b)
    only_b = _vjp(B, CL, CR, W, V, want_dC=False)
    assert only_b[1] is None and np.array_equal(only_b[0], full[0])
    only_c = _vjp(B, CL, CR, W, V, want_dB=False)
    assert only_c[0] is None and np.array_equal(only_c[1], full[1]) and np.array_equal(only_c[2], full[2])


def test_vjp_dot_product_with_oracle_jvp():
    B, CL, CR, W, V = _prob(40, 12, 2, 4, 13)
    dB, dCL, dCR = _vjp(B, CL, CR, W, V)
    rng = np.random.default_rng(5)
    tB = rng.standard_normal(B.shape)
    tB = 0.5 * (tB + tB.transpose(0, 2, 1))
    tL = rng.standard_normal(CL.shape)
    tR = rng.standard_normal(CR.shape)
    dJ, dK = oracle.jvp(B, CL, CR, tB, tL, tR)
    lhs = np.vdot(W, dJ) + np.vdot(V, dK)
    rhs = np.vdot(dB, tB) + np.vdot(dCL, tL) + np.vdot(dCR, tR)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("nao,naux,nd,r", [(70, 11, 3, 7), (131, 21, 2, 20), (50, 30, 8, 5)])
def test_vjp_symmetric_densities(nao, naux, nd, r):
    # C_L and C_R one buffer: the X-only recomputation (Y = X) gives the
    # general path's adjoints bit for bit, and the oracle's for C_R = C_L.
    from paper_2608_06536_amd import jk
    B, CL, _, W, V = _prob(nao, naux, nd, r, 400 + nao)
    Bd, Ld, Wd, Vd = _dev(B, CL, W, V)
    sym = [_np(t) for t in jk.jk_vjp(Bd, Ld, Ld, Wd, Vd)]
    gen = [_np(t) for t in jk.jk_vjp(Bd, Ld, Ld.clone(), Wd, Vd)]
    torch.cuda.synchronize()
    for a, b in zip(sym, gen):
        assert np.array_equal(a, b)
    rB, rL, rR = oracle.vjp(B, CL, CL, W, V)
    assert rel_err(sym[0], rB) <= TOL
    assert rel_err(sym[1], rL) <= TOL
    assert rel_err(sym[2], rR) <= TOL


def test_autograd_shared_factor():
    # J, K of D = C C^T through one leaf C: its gradient is dC_L + dC_R.
    from paper_2608_06536_amd import jk
    B, CL, _, W, V = _prob(33, 9, 2, 4, 18)
    C = torch.from_numpy(CL).cuda().requires_grad_(True)
    Bd, Wd, Vd = _dev(B, W, V)
    J, K = jk.jk(Bd, C, C)
    ((Wd * J).sum() + (Vd * K).sum()).backward()
    _, rL, rR = oracle.vjp(B, CL, CL, W, V)
    assert rel_err(C.grad.cpu().numpy(), rL + rR) <= TOL


def test_vjp_self_adjoint_gpu_forward():
    # dC_L = (J[W] + K[V]) C_R and dC_R = (J[W] + K[V])^T C_L, with J[W] and
    # K[V] from the GPU forward itself (C_L = W, C_R = I).
    from paper_2608_06536_amd import jk
    B, CL, CR, W, V = _prob(96, 30, 2, 6, 14)
    _, dCL, dCR = _vjp(B, CL, CR, W, V, want_dB=False)
    I = np.broadcast_to(np.eye(96), W.shape).copy()
    Bd, Wd, Vd, Id = _dev(B, W, V, I)
    JW, _ = jk.jk_build(Bd, Wd, Id, want_k=False)
    _, KV = jk.jk_build(Bd, Vd, Id, want_j=False)
    G = (JW + KV).cpu().numpy()
    assert rel_err(dCL, np.einsum("kmn,kni->kmi", G, CR)) <= TOL
    assert rel_err(dCR, np.einsum("knm,kni->kmi", G, CL)) <= TOL


def test_autograd_and_gradcheck():
    from paper_2608_06536_amd import jk
    B, CL, CR, W, V = _prob(12, 5, 2, 3, 15)
    A = torch.from_numpy(B).cuda().requires_grad_(True)
    L = torch.from_numpy(CL).cuda().requires_grad_(True)
    R = torch.from_numpy(CR).cuda().requires_grad_(True)
    Wd, Vd = _dev(W, V)
    J, K = jk.jk(A, L, R)
    loss = (Wd * J).sum() + (Vd * K).sum()
    loss.backward()
    rB, rL, rR = oracle.vjp(B, CL, CR, W, V)
    assert rel_err(A.grad.cpu().numpy(), rB) <= TOL
    assert rel_err(L.grad.cpu().numpy(), rL) <= TOL
    assert rel_err(R.grad.cpu().numpy(), rR) <= TOL

    # gradcheck through the symmetrising wrapper B = (A + A^T)/2
    def f(A_, L_, R_):
        Bs = 0.5 * (A_ + A_.transpose(1, 2))
        return jk.jk(Bs.contiguous(), L_, R_)

    small = _prob(6, 3, 1, 2, 16)
    args = [torch.from_numpy(x).cuda().requires_grad_(True) for x in small[:3]]
    assert torch.autograd.gradcheck(f, args, eps=1e-6, atol=1e-8, rtol=1e-7)


def test_config4_vjp_sampled():
    # Full differentiated workload (nao=500, naux=2000, nd=8, r=40) in the
    # benchmark's launch configuration: dB entries one by one, dC of one
    # density in full, and exact central differences through the GPU forward.
    from paper_2608_06536_amd import jk
    p = synth.config(4)
    B, CL, CR = synth.make_problem(p)
    W, V = synth.make_cotangents(p)
    Bd, Ld, Rd, Wd, Vd = _dev(B, CL, CR, W, V)
    dB, dCL, dCR = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    n = 16
    qs = rng.integers(0, p.naux, n)
    as_ = rng.integers(0, p.nao, n)
    bs = rng.integers(0, p.nao, n)
    as_[:3] = p.nao - 1
    qs[3] = p.naux - 1
    ref = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs)
    got = dB[qs, as_, bs].cpu().numpy()
    scale = float(dB.abs().max())
    assert np.max(np.abs(got - ref)) <= TOL * scale
    k = 5
    rl, rr = oracle.dc_density(B, CL[k], CR[k], W[k], V[k])
    assert rel_err(dCL[k].cpu().numpy(), rl) <= TOL
    assert rel_err(dCR[k].cpu().numpy(), rr) <= TOL

    # central differences: L is linear in C, so any step is exact up to rounding
    def loss(Bx, Lx, Rx):
        J, K = jk.jk_build(Bx, Lx, Rx)
        return float((Wd * J).sum() + (Vd * K).sum())

    for (kk, m, i) in [(0, 0, 0), (7, 499, 39), (3, 250, 17)]:
        for h in (1e-5, 1.0):
            E = torch.zeros_like(Ld)
            E[kk, m, i] = h
            fd = (loss(Bd, Ld + E, Rd) - loss(Bd, Ld - E, Rd)) / (2 * h)
            an = float(dCL[kk, m, i])
            # rounding of the loss difference bounds the agreement
            tol = 1e-9 if h == 1.0 else 1e-4
            assert abs(fd - an) <= tol * max(1.0, float(dCL.abs().max()))
