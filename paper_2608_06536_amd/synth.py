"""Seeded synthetic inputs for the Cholesky-decomposed J/K build.

This module draws random numbers and shapes arrays; it performs none of the
J/K arithmetic.  Both the GPU path's tests/benchmark and the CPU oracle's tests
take their inputs from here.

Workload recipe (stand-in for the paper's molecular Cholesky factors, which
are not available; sizes follow the paper's 236-472 AO series, Sec. 5.6, up
to 1000 AO):

* ``B^Q_mn = G^Q_mn * exp(-|m-n|/ell) * exp(-Q/tau)`` with ``G^Q`` standard
  normal on the upper triangle (diagonal included, row-major order) and
  mirrored, so every slab is exactly symmetric.  Slab ``Q`` is drawn from its
  own stream ``SeedSequence(seed, spawn_key=(0, Q))`` so any subset of slabs
  can be regenerated alone.
* Factor pairs ``C = orth(N(0,1) nao x r) @ N(0,1) r x r`` where ``orth`` is
  the Q factor of a QR decomposition with signs fixed so ``diag(R) > 0``.
  A "ground" density uses ``C_L = C_R = orth(...)`` (a projector); a
  "transition" density uses independent ``C_L`` and ``C_R``.
* Cotangents ``W``, ``V`` are standard normal ``nao x nao`` (non-symmetric).
* Laplace pseudo-density inputs (stand-in for SCF orbitals): coefficients
  ``C = orth(N(0,1) nao x (nocc + nvir))`` split into occupied and virtual
  columns; occupied energies: ``ncore`` core levels uniform in
  [-20.6, -11.0] Hartree, the rest valence levels uniform in [-1.4, -0.35];
  virtual energies log-uniform in [0.1, 20]; amplitudes ``X_m`` standard
  normal ``nocc x nvir``.  Energies are sorted ascending.
"""
from __future__ import annotations

import dataclasses
import functools
import os

import numpy as np

__all__ = [
    "Problem", "CONFIGS", "config", "make_B", "make_B_slabs", "make_B_parallel", "make_B_device",
    "make_factors",
    "make_cotangents", "make_problem", "batched_problems", "Orbitals", "make_orbitals",
    "make_amplitudes", "LAPLACE_BENCH",
]


@dataclasses.dataclass(frozen=True)
class Problem:
    """Shapes and generator parameters of one J/K problem."""
    nao: int
    naux: int
    nd: int
    r: int
    ell: float
    tau: float
    n_ground: int = 0      # number of leading ground (C_L = C_R) densities
    seed: int = 1000

    @property
    def rank(self) -> int:
        return self.nd * self.r

    def fwd_flops(self) -> float:
        """Algorithmic flops of one build: half-transforms 4, K 2, J 2."""
        return (6.0 * self.naux * self.nao ** 2 * self.rank
                + 2.0 * self.naux * self.nao ** 2 * self.nd)

    def vjp_flops(self) -> float:
        return 18.0 * self.naux * self.nao ** 2 * self.rank + 4.0 * self.naux * self.nao ** 2 * self.nd


# The five workloads (densities per config: config 2 is one ground plus three
# transition densities; config 4 and 5 are all transition densities).
CONFIGS = {
    1: Problem(nao=48, naux=192, nd=1, r=8, ell=8.0, tau=64.0, n_ground=0, seed=1001),
    2: Problem(nao=300, naux=1200, nd=4, r=30, ell=20.0, tau=300.0, n_ground=1, seed=1002),
    4: Problem(nao=500, naux=2000, nd=8, r=40, ell=20.0, tau=500.0, n_ground=0, seed=1004),
    5: Problem(nao=1000, naux=4000, nd=16, r=80, ell=20.0, tau=1000.0, n_ground=0, seed=1005),
}


def config(i: int) -> Problem:
    return CONFIGS[i]


@functools.lru_cache(maxsize=8)
def _slab_consts(nao: int, ell: float):
    """Upper-triangle indices and the decay matrix exp(-|m-n|/ell) (shared by
    every slab of a problem; read-only)."""
    iu = np.triu_indices(nao)
    idx = np.arange(nao)
    decay = np.exp(-np.abs(idx[:, None] - idx[None, :]) / ell)
    for a in (*iu, decay):
        a.setflags(write=False)
    return iu, decay


def _slab(nao: int, q: int, ell: float, tau: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(0, q)))
    iu, decay = _slab_consts(nao, ell)
    g = np.empty((nao, nao))
    g[iu] = rng.standard_normal(iu[0].size)
    g.T[iu] = g[iu]
    return g * decay * np.exp(-q / tau)


def make_B_slabs(p: Problem, qs, out: np.ndarray | None = None) -> np.ndarray:
    """Slabs ``B^Q`` for the listed Q values, shape ``[len(qs)][nao][nao]``."""
    qs = list(qs)
    if out is None:
        out = np.empty((len(qs), p.nao, p.nao))
    for j, q in enumerate(qs):
        out[j] = _slab(p.nao, q, p.ell, p.tau, p.seed)
    return out


def make_B(p: Problem) -> np.ndarray:
    """Full factor ``B[naux][nao][nao]`` (FP64, each slab symmetric)."""
    return make_B_slabs(p, range(p.naux))


def make_B_parallel(p: Problem, workers: int = 16, step: int = 32) -> np.ndarray:
    """``make_B(p)`` drawn by a pool of threads over blocks of slabs (each slab
    has its own stream, so the result is the same array)."""
    from concurrent.futures import ThreadPoolExecutor
    B = np.empty((p.naux, p.nao, p.nao))
    workers = max(1, min(workers, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda a: make_B_slabs(p, range(a, min(a + step, p.naux)),
                                           out=B[a:min(a + step, p.naux)]),
                    range(0, p.naux, step)))
    return B


def make_B_device(p: Problem, device):
    """The make_B recipe drawn on a GPU from torch's seeded generator: the
    same distribution and structure (symmetric slabs, exp(-|m-n|/ell) decay
    across a slab, exp(-Q/tau) across slabs), a different random stream from
    the host generator.  For timing batches too large to draw on the host;
    parity tests use make_B."""
    import torch
    g = torch.Generator(device=device).manual_seed(p.seed)
    B = torch.randn((p.naux, p.nao, p.nao), generator=g, dtype=torch.float64, device=device)
    B = torch.triu(B) + torch.triu(B, 1).transpose(1, 2)
    idx = torch.arange(p.nao, device=device, dtype=torch.float64)
    B *= torch.exp(-(idx[:, None] - idx[None, :]).abs() / p.ell)
    B *= torch.exp(-torch.arange(p.naux, device=device, dtype=torch.float64) / p.tau)[:, None, None]
    return B.contiguous()


def _orth(rng: np.random.Generator, nao: int, r: int) -> np.ndarray:
    m = rng.standard_normal((nao, r))
    q, rr = np.linalg.qr(m)
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s[None, :]


def make_factors(p: Problem) -> tuple[np.ndarray, np.ndarray]:
    """``C_L, C_R`` of shape ``[nd][nao][r]``."""
    rng = np.random.default_rng(np.random.SeedSequence(p.seed, spawn_key=(1,)))
    CL = np.empty((p.nd, p.nao, p.r))
    CR = np.empty((p.nd, p.nao, p.r))
    for k in range(p.nd):
        if k < p.n_ground:
            q0 = _orth(rng, p.nao, p.r)
            CL[k] = q0
            CR[k] = q0
        else:
            CL[k] = _orth(rng, p.nao, p.r) @ rng.standard_normal((p.r, p.r))
            CR[k] = _orth(rng, p.nao, p.r) @ rng.standard_normal((p.r, p.r))
    return CL, CR


def make_cotangents(p: Problem) -> tuple[np.ndarray, np.ndarray]:
    """``W, V`` of shape ``[nd][nao][nao]``, standard normal."""
    rng = np.random.default_rng(np.random.SeedSequence(p.seed, spawn_key=(2,)))
    W = rng.standard_normal((p.nd, p.nao, p.nao))
    V = rng.standard_normal((p.nd, p.nao, p.nao))
    return W, V


def make_problem(p: Problem):
    """``(B, CL, CR)`` for problem ``p``."""
    B = make_B(p)
    CL, CR = make_factors(p)
    return B, CL, CR


def batched_problems(n_geom: int = 64, lo: int = 100, hi: int = 500,
                     seed: int = 1003, nd: int = 6, nao_list=None) -> list[Problem]:
    """The uneven batched workload: ``n_geom`` geometries with nao drawn
    uniformly from the integers in [lo, hi], naux = 4 nao, nd densities (one
    ground, the rest transition) of rank floor(nao/10), ell = 20,
    tau = naux/4."""
    if nao_list is None:
        rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(3,)))
        nao_list = rng.integers(lo, hi, size=n_geom, endpoint=True)
    out = []
    for g, nao in enumerate(nao_list):
        nao = int(nao)
        naux = 4 * nao
        out.append(Problem(nao=nao, naux=naux, nd=nd, r=max(1, nao // 10), ell=20.0,
                           tau=naux / 4.0, n_ground=1, seed=seed * 1000 + g))
    return out


@dataclasses.dataclass(frozen=True)
class Orbitals:
    """Shapes and generator parameters of one set of synthetic orbitals."""
    nao: int
    nocc: int
    nvir: int
    ncore: int = 0
    seed: int = 2000


def make_orbitals(o: Orbitals):
    """``(Cocc [nao][nocc], e_occ [nocc], Cvir [nao][nvir], e_vir [nvir])``."""
    rng = np.random.default_rng(np.random.SeedSequence(o.seed, spawn_key=(4,)))
    C = _orth(rng, o.nao, o.nocc + o.nvir)
    core = rng.uniform(-20.6, -11.0, size=o.ncore)
    val = rng.uniform(-1.4, -0.35, size=o.nocc - o.ncore)
    e_occ = np.sort(np.concatenate([core, val]))
    e_vir = np.sort(0.1 * 200.0 ** rng.uniform(0.0, 1.0, size=o.nvir))
    return (np.ascontiguousarray(C[:, :o.nocc]), e_occ,
            np.ascontiguousarray(C[:, o.nocc:]), e_vir)


def make_amplitudes(o: Orbitals, nvec: int) -> np.ndarray:
    """``X [nvec][nocc][nvir]``, standard normal."""
    rng = np.random.default_rng(np.random.SeedSequence(o.seed, spawn_key=(5,)))
    return rng.standard_normal((nvec, o.nocc, o.nvir))


# The Laplace driver's benchmark: the differentiated-build sizes (nao = 500,
# naux = 2000) with nocc = 40 occupied orbitals (8 of them core), the other
# 460 columns virtual, one amplitude matrix and 8 quadrature points, so the
# build sees 8 transition densities of rank 40.
LAPLACE_BENCH = (Orbitals(nao=500, nocc=40, nvir=460, ncore=8, seed=2004), 1, 8)
