"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own formulas:

* a hand-worked 2x2 example (tests/golden);
* brute force through the explicit 4-index tensor (mn|ls) = sum_Q B^Q_mn B^Q_ls
  (the definition of the Cholesky-decomposed integrals, Sec. 2.3);
* closed forms for special factors (identity, rank-1, diagonal slabs);
* invariants of Eq. (4): K[D^T] = K[D]^T, J depends on sym(D) only,
  linearity, self-adjointness (Eq. (1)), energies from r x r matrices,
  gauge and Q-permutation invariance, Q-blocking independence;
* derivatives: central differences (exact here, because the scalar is linear
  in C_L and C_R and quadratic in B), a dot-product test between the
  reverse- and forward-mode derivatives, and the self-adjoint identity
  dC_L = (J[W] + K[V]) C_R built from forward calls.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a transposed operand, a wrong index) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2608_06536_amd import synth
from conftest import rel_err

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(seed, nao, naux, nd, r, sym=True):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((naux, nao, nao))
    if sym:
        B = 0.5 * (B + B.transpose(0, 2, 1))
    CL = rng.standard_normal((nd, nao, r))
    CR = rng.standard_normal((nd, nao, r))
    return B, CL, CR


# ------------------------------------------------------------------ worked example

def test_handworked_2x2():
    g = json.load(open(os.path.join(GOLD, "handworked_2x2.json")))
    B = np.array(g["B"], float)
    CL = np.array(g["CL"], float)
    CR = np.array(g["CR"], float)
    D = oracle.density(CL, CR)
    assert np.array_equal(D, np.array(g["D"], float))
    J1, K1 = oracle.jk_plain(B, CL, CR)
    J2, K2, gam = oracle.jk_factored(B, CL, CR)
    assert np.array_equal(gam, np.array(g["gamma"], float))
    for J in (J1, J2):
        assert np.array_equal(J, np.array(g["J"], float))
    for K in (K1, K2):
        assert np.array_equal(K, np.array(g["K"], float))
    eri = oracle.eri4(B)
    J0, K0 = oracle.jk_from_eri(eri, D[0])
    assert np.array_equal(J0, np.array(g["J"], float)[0])
    assert np.array_equal(K0, np.array(g["K"], float)[0])


# ------------------------------------------------------------------ brute force

def test_bruteforce_config1():
    p = synth.config(1)
    B, CL, CR = synth.make_problem(p)
    D = oracle.density(CL, CR)
    eri = oracle.eri4(B)
    J0, K0 = oracle.jk_from_eri(eri, D[0])
    J1, K1 = oracle.jk_plain(B, CL, CR)
    J2, K2, _ = oracle.jk_factored(B, CL, CR)
    assert rel_err(J1[0], J0) < 1e-13 and rel_err(K1[0], K0) < 1e-13
    assert rel_err(J2[0], J0) < 1e-13 and rel_err(K2[0], K0) < 1e-13


@pytest.mark.parametrize("seed,nao,naux", [(1, 5, 3), (2, 11, 7), (3, 24, 9), (4, 1, 2)])
def test_bruteforce_general_B(seed, nao, naux):
    # Non-symmetric slabs and a non-factored density: the plain definition (T1)
    # must still equal the 4-index contraction.
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((naux, nao, nao))
    D = rng.standard_normal((1, nao, nao))
    eri = oracle.eri4(B)
    J0, K0 = oracle.jk_from_eri(eri, D[0])
    J1, K1 = oracle.jk_from_density(B, D)
    assert rel_err(J1[0], J0) < 1e-13
    assert rel_err(K1[0], K0) < 1e-13


@pytest.mark.parametrize("seed,nao,naux,nd,r", [(5, 17, 6, 3, 4), (6, 24, 10, 2, 7), (7, 9, 1, 1, 9)])
def test_factored_equals_plain(seed, nao, naux, nd, r):
    B, CL, CR = _rand_problem(seed, nao, naux, nd, r)
    J1, K1 = oracle.jk_plain(B, CL, CR)
    J2, K2, g = oracle.jk_factored(B, CL, CR)
    assert rel_err(J2, J1) < 1e-13 and rel_err(K2, K1) < 1e-13
    assert rel_err(g, oracle.project(B, oracle.density(CL, CR))) < 1e-13


# ------------------------------------------------------------------ closed forms

def test_identity_slabs():
    # B^Q = I for all Q:  K = naux D,  J = naux tr(D) I.
    nao, naux = 13, 5
    rng = np.random.default_rng(8)
    B = np.broadcast_to(np.eye(nao), (naux, nao, nao)).copy()
    CL = rng.standard_normal((2, nao, 3))
    CR = rng.standard_normal((2, nao, 3))
    D = np.einsum("kmi,kni->kmn", CL, CR)
    J, K, _ = oracle.jk_factored(B, CL, CR)
    J1, K1 = oracle.jk_plain(B, CL, CR)
    for k in range(2):
        tr = np.trace(D[k])
        assert rel_err(K[k], naux * D[k]) < 1e-14
        assert rel_err(J[k], naux * tr * np.eye(nao)) < 1e-14
        assert rel_err(K1[k], naux * D[k]) < 1e-14
        assert rel_err(J1[k], naux * tr * np.eye(nao)) < 1e-14


def test_rank1_slabs_give_J_equal_K():
    # B^Q = b_Q b_Q^T:  J_mn = sum_Q (b^T D b) b_m b_n = K_mn for any D.
    nao, naux = 10, 6
    rng = np.random.default_rng(9)
    b = rng.standard_normal((naux, nao))
    B = np.einsum("qm,qn->qmn", b, b)
    D = rng.standard_normal((1, nao, nao))
    J, K = oracle.jk_from_density(B, D)
    assert rel_err(J, K) < 1e-14
    CL = rng.standard_normal((1, nao, 4))
    CR = rng.standard_normal((1, nao, 4))
    J2, K2, _ = oracle.jk_factored(B, CL, CR)
    assert rel_err(J2, K2) < 1e-14


def test_diagonal_slabs():
    # B^Q = diag(b_Q):  K_mn = sum_Q b_Qm D_mn b_Qn,  J = diag(sum_Q (b_Q . diag D) b_Q).
    nao, naux = 9, 4
    rng = np.random.default_rng(10)
    b = rng.standard_normal((naux, nao))
    B = np.zeros((naux, nao, nao))
    for q in range(naux):
        B[q] = np.diag(b[q])
    D = rng.standard_normal((1, nao, nao))
    J, K = oracle.jk_from_density(B, D)
    Kx = np.zeros((nao, nao))
    Jd = np.zeros(nao)
    for q in range(naux):
        Kx += np.outer(b[q], b[q]) * D[0]
        Jd += (b[q] * np.diag(D[0])).sum() * b[q]
    assert rel_err(K[0], Kx) < 1e-14
    assert rel_err(J[0], np.diag(Jd)) < 1e-14


def test_rank_one_density_outer_products():
    # nd = 1, r = 1: K = sum_Q (B^Q c_L)(B^Q c_R)^T, a sum of outer products.
    nao, naux = 12, 5
    B, CL, CR = _rand_problem(11, nao, naux, 1, 1)
    _, K = oracle.jk_plain(B, CL, CR)
    Kx = sum(np.outer(B[q] @ CL[0, :, 0], B[q] @ CR[0, :, 0]) for q in range(naux))
    assert rel_err(K[0], Kx) < 1e-14


# ------------------------------------------------------------------ invariants

@pytest.fixture(scope="module")
def small():
    return _rand_problem(12, 20, 8, 3, 5)


def test_transpose_rules(small):
    B, CL, CR = small
    J, K, _ = oracle.jk_factored(B, CL, CR)
    Jt, Kt, _ = oracle.jk_factored(B, CR, CL)  # D -> D^T
    assert rel_err(Kt, K.transpose(0, 2, 1)) < 1e-14
    assert rel_err(Jt, J) < 1e-14
    assert rel_err(J, J.transpose(0, 2, 1)) < 1e-14


def test_J_sees_only_symmetric_part():
    nao, naux = 14, 6
    rng = np.random.default_rng(13)
    B = rng.standard_normal((naux, nao, nao))
    B = 0.5 * (B + B.transpose(0, 2, 1))
    A = rng.standard_normal((1, nao, nao))
    anti = A - A.transpose(0, 2, 1)
    J, K = oracle.jk_from_density(B, anti)
    assert np.max(np.abs(J)) < 1e-12
    assert np.max(np.abs(K)) > 1e-3   # the antisymmetric part still reaches K


def test_linearity_in_density(small):
    B, CL, CR = small
    # D1 + D2 by concatenating ranks: [C1 | C2] [C1' | C2']^T
    J1, K1, _ = oracle.jk_factored(B, CL[:1], CR[:1])
    J2, K2, _ = oracle.jk_factored(B, CL[1:2], CR[1:2])
    CLc = np.concatenate([CL[:1], 2.5 * CL[1:2]], axis=2)
    CRc = np.concatenate([CR[:1], CR[1:2]], axis=2)
    J12, K12, _ = oracle.jk_factored(B, CLc, CRc)
    assert rel_err(J12, J1 + 2.5 * J2) < 1e-13
    assert rel_err(K12, K1 + 2.5 * K2) < 1e-13


def test_self_adjoint(small):
    # <D1, J[D2]> = <J[D1], D2> and the same for K (Eq. (1)); this is the
    # invariance of the scalar under W_L <-> W_R (Sec. 2.3).
    B = small[0]
    nao = B.shape[1]
    rng = np.random.default_rng(14)
    D1 = rng.standard_normal((1, nao, nao))
    D2 = rng.standard_normal((1, nao, nao))
    J1, K1 = oracle.jk_from_density(B, D1)
    J2, K2 = oracle.jk_from_density(B, D2)
    a, b = np.vdot(D1, J2), np.vdot(J1, D2)
    assert abs(a - b) < 1e-12 * abs(a)
    a, b = np.vdot(D1, K2), np.vdot(K1, D2)
    assert abs(a - b) < 1e-12 * abs(a)


def test_energies_from_small_matrices(small):
    B, CL, CR = small
    J, K, g = oracle.jk_factored(B, CL, CR)
    D = np.einsum("kmi,kni->kmn", CL, CR)
    for k in range(CL.shape[0]):
        eJ = sum(np.trace(CR[k].T @ B[q] @ CL[k]) ** 2 for q in range(B.shape[0]))
        eK = sum(np.vdot(CL[k].T @ B[q] @ CL[k], CR[k].T @ B[q] @ CR[k]) for q in range(B.shape[0]))
        assert np.vdot(D[k], J[k]) >= 0.0
        assert abs(np.vdot(D[k], J[k]) - eJ) < 1e-12 * abs(eJ)
        assert abs(np.vdot(D[k], K[k]) - eK) < 1e-12 * abs(eK)


def test_gauge_invariance(small):
    B, CL, CR = small
    rng = np.random.default_rng(15)
    r = CL.shape[2]
    G = rng.standard_normal((r, r)) + 3 * np.eye(r)
    CLg = CL @ G
    CRg = CR @ np.linalg.inv(G).T
    J, K, _ = oracle.jk_factored(B, CL, CR)
    Jg, Kg, _ = oracle.jk_factored(B, CLg, CRg)
    assert rel_err(Jg, J) < 1e-12 and rel_err(Kg, K) < 1e-12


def test_q_permutation_and_blocking(small):
    B, CL, CR = small
    J, K, _ = oracle.jk_factored(B, CL, CR)
    perm = np.random.default_rng(16).permutation(B.shape[0])
    Jp, Kp, _ = oracle.jk_factored(B[perm], CL, CR)
    assert rel_err(Jp, J) < 1e-14 and rel_err(Kp, K) < 1e-14
    h = 3
    Ja, Ka, _ = oracle.jk_factored(B[:h], CL, CR)
    Jb, Kb, _ = oracle.jk_factored(B[h:], CL, CR)
    assert rel_err(Ja + Jb, J) < 1e-14 and rel_err(Ka + Kb, K) < 1e-14


def test_scaling_of_B(small):
    B, CL, CR = small
    J, K, _ = oracle.jk_factored(B, CL, CR)
    J3, K3, _ = oracle.jk_factored(3.0 * B, CL, CR)
    assert rel_err(J3, 9.0 * J) < 1e-14 and rel_err(K3, 9.0 * K) < 1e-14


def test_entries_match_full(small):
    B, CL, CR = small
    J, K, _ = oracle.jk_factored(B, CL, CR)
    rng = np.random.default_rng(17)
    n = 12
    ks = rng.integers(0, CL.shape[0], n)
    ms = rng.integers(0, B.shape[1], n)
    ns = rng.integers(0, B.shape[1], n)
    Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms, ns)
    scale_j, scale_k = np.max(np.abs(J)), np.max(np.abs(K))
    assert np.max(np.abs(Je - J[ks, ms, ns])) < 1e-13 * scale_j
    assert np.max(np.abs(Ke - K[ks, ms, ns])) < 1e-13 * scale_k


# ------------------------------------------------------------------ derivatives

def _loss(B, CL, CR, W, V):
    J, K = oracle.jk_plain(B, CL, CR)
    return float(np.vdot(W, J) + np.vdot(V, K))


@pytest.fixture(scope="module")
def dprob():
    B, CL, CR = _rand_problem(20, 9, 4, 2, 3)
    rng = np.random.default_rng(21)
    W = rng.standard_normal((2, 9, 9))
    V = rng.standard_normal((2, 9, 9))
    return B, CL, CR, W, V


@pytest.mark.parametrize("general", [False, True])
def test_vjp_central_differences_factors(dprob, general):
    # L is linear in C_L and in C_R separately: central differences are exact
    # up to rounding for any step.  Also with a non-symmetric B, where the
    # transposes in dL/dD = sum omega B + B^T V B^T matter.
    B, CL, CR, W, V = dprob
    if general:
        B = B + 0.3 * np.random.default_rng(27).standard_normal(B.shape)
    _, dCL, dCR = oracle.vjp(B, CL, CR, W, V, want_dB=False)
    h = 0.25
    scale = np.max(np.abs(dCL)) + np.max(np.abs(dCR))
    for idx in [(0, 0, 0), (1, 3, 2), (0, 8, 1), (1, 5, 0)]:
        E = np.zeros_like(CL)
        E[idx] = h
        fd = (_loss(B, CL + E, CR, W, V) - _loss(B, CL - E, CR, W, V)) / (2 * h)
        assert abs(fd - dCL[idx]) < 1e-12 * scale
        fd = (_loss(B, CL, CR + E, W, V) - _loss(B, CL, CR - E, W, V)) / (2 * h)
        assert abs(fd - dCR[idx]) < 1e-12 * scale


def test_vjp_central_differences_B_general(dprob):
    # L is quadratic in B: central differences are exact; perturb single
    # entries of a NON-symmetric B through the literal forward.
    B, CL, CR, W, V = dprob
    rng = np.random.default_rng(22)
    Bg = B + 0.3 * rng.standard_normal(B.shape)
    dB, _, _ = oracle.vjp(Bg, CL, CR, W, V)
    h = 0.5
    scale = np.max(np.abs(dB))
    for idx in [(0, 0, 0), (1, 2, 7), (3, 7, 2), (2, 4, 4), (0, 8, 1)]:
        E = np.zeros_like(Bg)
        E[idx] = h
        fd = (_loss(Bg + E, CL, CR, W, V) - _loss(Bg - E, CL, CR, W, V)) / (2 * h)
        assert abs(fd - dB[idx]) < 1e-12 * scale


def test_vjp_random_direction(dprob):
    B, CL, CR, W, V = dprob
    dB, dCL, dCR = oracle.vjp(B, CL, CR, W, V)
    rng = np.random.default_rng(23)
    for which in range(3):
        dirs = [np.zeros_like(B), np.zeros_like(CL), np.zeros_like(CR)]
        dirs[which] = rng.standard_normal(dirs[which].shape)
        args_p = [B + dirs[0], CL + dirs[1], CR + dirs[2]]
        args_m = [B - dirs[0], CL - dirs[1], CR - dirs[2]]
        fd = (_loss(*args_p, W, V) - _loss(*args_m, W, V)) / 2.0
        an = np.vdot(dB, dirs[0]) + np.vdot(dCL, dirs[1]) + np.vdot(dCR, dirs[2])
        assert abs(fd - an) < 1e-11 * max(1.0, abs(an))


def test_vjp_dot_product_with_jvp(dprob):
    # <(W,V), JVP(x)> = <VJP(W,V), x> for a joint direction (the transpose
    # check of Sec. 2.1).
    B, CL, CR, W, V = dprob
    rng = np.random.default_rng(24)
    tB = rng.standard_normal(B.shape)
    tL = rng.standard_normal(CL.shape)
    tR = rng.standard_normal(CR.shape)
    dJ, dK = oracle.jvp(B, CL, CR, tB, tL, tR)
    dB, dCL, dCR = oracle.vjp(B, CL, CR, W, V)
    lhs = np.vdot(W, dJ) + np.vdot(V, dK)
    rhs = np.vdot(dB, tB) + np.vdot(dCL, tL) + np.vdot(dCR, tR)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_jvp_central_differences(dprob):
    # J, K are quadratic in B and linear in each factor: per-argument central
    # differences reproduce the forward derivative exactly.
    B, CL, CR, _, _ = dprob
    rng = np.random.default_rng(25)
    for which in range(3):
        t = [None, None, None]
        shapes = [B.shape, CL.shape, CR.shape]
        t[which] = rng.standard_normal(shapes[which])
        dJ, dK = oracle.jvp(B, CL, CR, *t)
        p = [B, CL, CR]
        pp = [x + (t[i] if i == which else 0) for i, x in enumerate(p)]
        pm = [x - (t[i] if i == which else 0) for i, x in enumerate(p)]
        Jp, Kp = oracle.jk_plain(*pp)
        Jm, Km = oracle.jk_plain(*pm)
        assert rel_err(dJ, (Jp - Jm) / 2) < 1e-12
        assert rel_err(dK, (Kp - Km) / 2) < 1e-12


def test_vjp_self_adjoint_forward_reuse(dprob):
    # dC_L = (J[W] + K[V]) C_R and dC_R = (J[W] + K[V])^T C_L, with J[W], K[V]
    # from the FORWARD build (C_L = W, C_R = I): the adjoint reuses the
    # forward kernel (Eq. (1)).
    B, CL, CR, W, V = dprob
    nao = B.shape[1]
    _, dCL, dCR = oracle.vjp(B, CL, CR, W, V, want_dB=False)
    I = np.broadcast_to(np.eye(nao), W.shape).copy()
    JW, _, _ = oracle.jk_factored(B, W, I)
    _, KV, _ = oracle.jk_factored(B, V, I)
    G = JW + KV
    assert rel_err(dCL, np.einsum("kmn,kni->kmi", G, CR)) < 1e-13
    assert rel_err(dCR, np.einsum("knm,kni->kmi", G, CL)) < 1e-13


def test_vjp_symmetric_part_convention_free(dprob):
    # For symmetric B the symmetric part of dB equals the derivative along
    # symmetric perturbations (pairs B_ab, B_ba moved together).
    B, CL, CR, W, V = dprob
    dB, _, _ = oracle.vjp(B, CL, CR, W, V)
    h = 0.5
    for (q, a, b) in [(0, 1, 5), (2, 3, 3), (3, 8, 0)]:
        E = np.zeros_like(B)
        E[q, a, b] += h
        if a != b:
            E[q, b, a] += h
        fd = (_loss(B + E, CL, CR, W, V) - _loss(B - E, CL, CR, W, V)) / (2 * h)
        an = dB[q, a, b] + (dB[q, b, a] if a != b else 0.0)
        assert abs(fd - an) < 1e-12 * np.max(np.abs(dB))


def test_vjp_entry_and_density_forms(dprob):
    B, CL, CR, W, V = dprob
    dB, dCL, dCR = oracle.vjp(B, CL, CR, W, V)
    rng = np.random.default_rng(26)
    qs = rng.integers(0, B.shape[0], 10)
    as_ = rng.integers(0, B.shape[1], 10)
    bs = rng.integers(0, B.shape[1], 10)
    e = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs)
    assert np.max(np.abs(e - dB[qs, as_, bs])) < 1e-13 * np.max(np.abs(dB))
    for k in range(CL.shape[0]):
        dl, dr = oracle.dc_density(B, CL[k], CR[k], W[k], V[k])
        assert rel_err(dl, dCL[k]) < 1e-13 and rel_err(dr, dCR[k]) < 1e-13


def test_vjp_factored_equals_literal(dprob):
    # the factored derivative (the GPU's own arrangement) against the literal
    # closed forms, and its Q-range restriction against a Q-split sum
    B, CL, CR, W, V = dprob
    rB, rL, rR = oracle.vjp(B, CL, CR, W, V)
    fB, fL, fR = oracle.vjp_factored(B, CL, CR, W, V)
    assert rel_err(fB, rB) < 1e-13 and rel_err(fL, rL) < 1e-13 and rel_err(fR, rR) < 1e-13
    aB, aL, aR = oracle.vjp_factored(B, CL, CR, W, V, 0, 2)
    bB, bL, bR = oracle.vjp_factored(B, CL, CR, W, V, 2, None)
    assert rel_err(aB + bB, fB) < 1e-14 and rel_err(aL + bL, fL) < 1e-14
    for Wx, Vx in ((W, None), (None, V)):
        rB, rL, rR = oracle.vjp(B, CL, CR, Wx, Vx)
        fB, fL, fR = oracle.vjp_factored(B, CL, CR, Wx, Vx)
        assert rel_err(fB, rB) < 1e-13 and rel_err(fL, rL) < 1e-13 and rel_err(fR, rR) < 1e-13


def test_vjp_factored_one_sided_outputs(dprob):
    # either factor adjoint alone (the other output NULL) equals its part of
    # the two-sided call, and no output is touched through a NULL pointer
    B, CL, CR, W, V = dprob
    _, fL, fR = oracle.vjp_factored(B, CL, CR, W, V, want_dB=False)
    _, oL, nR = oracle.vjp_factored(B, CL, CR, W, V, want_dB=False, want_dCR=False)
    _, nL, oR = oracle.vjp_factored(B, CL, CR, W, V, want_dB=False, want_dCL=False)
    assert nR is None and nL is None
    assert np.array_equal(oL, fL) and np.array_equal(oR, fR)


def test_vjp_zero_cotangents(dprob):
    B, CL, CR, W, V = dprob
    dB, dCL, dCR = oracle.vjp(B, CL, CR, None, None)
    assert not np.any(dB) and not np.any(dCL) and not np.any(dCR)
    dBw, dCLw, dCRw = oracle.vjp(B, CL, CR, W, None)
    dBv, dCLv, dCRv = oracle.vjp(B, CL, CR, None, V)
    dBb, dCLb, dCRb = oracle.vjp(B, CL, CR, W, V)
    assert rel_err(dBw + dBv, dBb) < 1e-14
    assert rel_err(dCLw + dCLv, dCLb) < 1e-14


# ------------------------------------------------------------------ generator

def test_generator_properties():
    p = synth.config(1)
    B, CL, CR = synth.make_problem(p)
    assert B.shape == (p.naux, p.nao, p.nao) and CL.shape == (p.nd, p.nao, p.r)
    assert np.array_equal(B, B.transpose(0, 2, 1))
    B2 = synth.make_B_slabs(p, [5, 77])
    assert np.array_equal(B2[0], B[5]) and np.array_equal(B2[1], B[77])
    B3, CL3, CR3 = synth.make_problem(p)
    assert np.array_equal(B, B3) and np.array_equal(CL, CL3) and np.array_equal(CR, CR3)
    p2 = synth.config(2)
    CL2, CR2 = synth.make_factors(p2)
    # ground density: C_L = C_R with orthonormal columns (D is a projector)
    assert np.array_equal(CL2[0], CR2[0])
    assert np.allclose(CL2[0].T @ CL2[0], np.eye(p2.r), atol=1e-12)
    assert not np.array_equal(CL2[1], CR2[1])
