"""CPU pins of the Laplace oracle (Sec. 2.2, Eq. (laplace)).

The oracle's rule is pinned by what fixes the best approximation: the
one-term closed form and the alternation theorem (2n + 1 alternating, level
extrema on an independent dense scan).  Its written-out definitions are
pinned against each other and against the already pinned J/K oracle: the
pseudo-density sum reproduces the elementwise MO formula, the quadrature
contractions stay within the rigorous bound E * sum |integral * X| / x of
the exact ones (and not vacuously), the MO integrals match the four-index
oracle, and the AO route (J/K builds on the scaled factors, projected on the
orbitals) reproduces the MO route.
"""
import numpy as np
import pytest

import oracle
from oracle import laplace as OL
from paper_2608_06536_amd import synth


def scan_extrema(w, a, R, m=400001):
    """Independent dense scan: the maximum |eta| and the alternating extrema."""
    y = np.exp(np.linspace(0.0, np.log(R), m))
    e = OL.relative_error(w, a, y)
    idx = [0] + [i for i in range(1, m - 1) if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) < 0] + [m - 1]
    ext = []
    for i in idx:
        if ext and (ext[-1] > 0) == (e[i] > 0):
            if abs(e[i]) > abs(ext[-1]):
                ext[-1] = e[i]
        else:
            ext.append(e[i])
    return float(np.max(np.abs(e))), np.array(ext)


def oracle_rule(n, x_min, x_max):
    w, a, E, lev = OL.minimax_rule(n, x_max / x_min)
    return w / x_min, a / x_min, E, lev


@pytest.mark.parametrize("R", [2.0, 10.0, 87.0, 1e4, 1e6])
def test_oracle_one_term_closed_form(R):
    w0, a0, E0 = OL.closed_form_one_term(R)
    # the closed form itself: three alternating, level extrema at 1, 1/a, R
    e = OL.relative_error([w0], [a0], [1.0, 1.0 / a0, R])
    assert np.allclose(e, [E0, -E0, E0], rtol=1e-12, atol=0)
    wo, ao, Eo, levo = OL.minimax_rule(1, R)
    assert levo and abs(ao[0] / a0 - 1) < 1e-10 and abs(wo[0] / w0 - 1) < 1e-10
    assert abs(Eo / E0 - 1) < 1e-9


@pytest.mark.parametrize("n,R", [(2, 10.0), (4, 100.0), (6, 100.0), (8, 1e3), (10, 1e3)])
def test_oracle_rule_equioscillates(n, R):
    w, a, E, lev = OL.minimax_rule(n, R)
    assert lev and np.all(w > 0) and np.all(a > 0)
    mx, ext = scan_extrema(w, a, R)
    assert ext.size == 2 * n + 1
    mags = np.abs(ext)
    assert (mags.max() - mags.min()) <= 1e-4 * mags.max()
    assert E * (1 - 1e-4) <= mx <= E * (1 + 1e-12)


# ---------------------------------------------------------------- the oracle
def _orbitals(nao=12, nocc=3, nvir=5, ncore=1, seed=11, nvec=2):
    o = synth.Orbitals(nao=nao, nocc=nocc, nvir=nvir, ncore=ncore, seed=seed)
    Co, eo, Cv, ev = synth.make_orbitals(o)
    X = synth.make_amplitudes(o, nvec)
    p = synth.Problem(nao=nao, naux=7, nd=1, r=1, ell=4.0, tau=3.0, seed=seed)
    return synth.make_B(p), Co, eo, Cv, ev, X


def test_scaled_factors_special_cases():
    _, Co, eo, Cv, ev, X = _orbitals()
    # alpha = 0: a plain product with X^T, weighted
    f = OL.scaled_factors(Cv, ev, np.zeros(2), np.array([1.0, 3.0]), -1.0, X=X)
    for m in range(X.shape[0]):
        assert np.allclose(f[0, m], Cv @ X[m].T, rtol=0, atol=1e-14)
        assert np.allclose(f[1, m], 3.0 * Cv @ X[m].T, rtol=0, atol=1e-14)
    # no X: column scaling, the same for every m
    f = OL.scaled_factors(Co, eo, np.array([0.7]), np.array([2.0]), 0.5, nvec=3)
    for m in range(3):
        for i in range(Co.shape[1]):
            assert np.allclose(f[0, m][:, i], 2.0 * Co[:, i] * np.exp(0.35 * eo[i]), rtol=1e-15)


def test_pseudo_density_sum_is_mo_formula():
    # sum_k CL_k CR_k^T = Cocc [X o q(e_b - e_j + shift)] Cvir^T elementwise in
    # the orbital indices, q(x) = sum_k w_k exp(-alpha_k x)
    _, Co, eo, Cv, ev, X = _orbitals()
    w = np.array([0.3, 1.1, 2.0])
    al = np.array([0.05, 0.4, 1.7])
    shift = 0.3
    CL = OL.scaled_factors(Co, eo, al, w * np.exp(-al * shift), +1.0, nvec=X.shape[0])
    CR = OL.scaled_factors(Cv, ev, al, np.ones(3), -1.0, X=X)
    x = ev[None, :] - eo[:, None] + shift
    q = OL.quadrature_of(w, al, x)
    for m in range(X.shape[0]):
        lhs = sum(CL[k, m] @ CR[k, m].T for k in range(3))
        rhs = Co @ (X[m] * q) @ Cv.T
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-13 * np.max(np.abs(rhs)))


def test_mo_eri_matches_four_index_oracle():
    B, Co, eo, Cv, ev, X = _orbitals()
    eri = oracle.eri4(B)                      # (mn|ls), pinned elsewhere by brute force
    ref = np.einsum("mp,nq,lr,tu,mnlt->pqru", Co, Cv, Co, Cv, eri)
    got = OL.mo_eri(B, Co, Cv, Co, Cv)
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


@pytest.mark.parametrize("shift", [0.0, 0.25])
def test_contractions_within_quadrature_bound(shift):
    B, Co, eo, Cv, ev, X = _orbitals()
    Xm = X[0]
    for fn, k in ((OL.pair_contraction, 1), (OL.doubles_contraction, 2)):
        lo = k * (ev.min() - eo.max()) + shift
        hi = k * (ev.max() - eo.min()) + shift
        for n in (4, 8):
            w, a, E, _ = oracle_rule(n, lo, hi)
            sJ, sK, bJ, bK = fn(B, Co, eo, Cv, ev, Xm, shift)
            qJ, qK, _, _ = fn(B, Co, eo, Cv, ev, Xm, shift, rule=(w, a))
            assert np.all(np.abs(qJ - sJ) <= E * bJ * (1 + 1e-9) + 1e-15)
            assert np.all(np.abs(qK - sK) <= E * bK * (1 + 1e-9) + 1e-15)
            # and the bound is not vacuous: the error is a visible fraction of it
            assert np.max(np.abs(qJ - sJ)) > 1e-3 * E * np.max(bJ)


def test_ao_route_equals_mo_route():
    # J/K builds (the pinned C oracle) on the scaled factors, projected on the
    # orbitals and rescaled, reproduce the quadrature contractions
    B, Co, eo, Cv, ev, X = _orbitals(nvec=1)
    shift = 0.1
    w = np.array([0.02, 0.3, 1.5, 4.0])
    al = np.array([0.01, 0.2, 0.9, 3.0])
    CL = OL.scaled_factors(Co, eo, al, w * np.exp(-al * shift), +1.0, nvec=1)
    CR = OL.scaled_factors(Cv, ev, al, np.ones(4), -1.0, X=X)
    J, K, _ = oracle.jk_factored(B, CL[:, 0].copy(), CR[:, 0].copy())
    # one excitation: sum over k, then project
    pJ, pK, _, _ = OL.pair_contraction(B, Co, eo, Cv, ev, X[0], shift, rule=(w, al))
    assert np.allclose(Co.T @ J.sum(0) @ Cv, pJ, rtol=0, atol=1e-12 * np.max(np.abs(pJ)))
    assert np.allclose(Co.T @ K.sum(0) @ Cv, pK, rtol=0, atol=1e-12 * np.max(np.abs(pK)))
    # two excitations: project each k, scale by exp(alpha_k (e_i - e_a)), sum
    dJ, dK, _, _ = OL.doubles_contraction(B, Co, eo, Cv, ev, X[0], shift, rule=(w, al))
    sc = np.exp(al[:, None, None] * (eo[None, :, None] - ev[None, None, :]))
    gJ = np.einsum("kia,mi,kmn,na->ia", sc, Co, J, Cv)
    gK = np.einsum("kia,mi,kmn,na->ia", sc, Co, K, Cv)
    assert np.allclose(gJ, dJ, rtol=0, atol=1e-12 * np.max(np.abs(dJ)))
    assert np.allclose(gK, dK, rtol=0, atol=1e-12 * np.max(np.abs(dK)))
