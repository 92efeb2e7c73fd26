"""Benchmark of the Cholesky-decomposed J/K path on one MI355X.

One step = one pass of the hot path over the differentiated workload
(nao=500, naux=2000, 8 non-symmetric densities of rank 40): the FP64 forward
build jk_build (gamma, J, half-transforms, K) followed by the reverse-mode
derivative jk_vjp with N(0,1) cotangents (dB, dC_L, dC_R).  Inputs are seeded
synthetic arrays resident on the GPU before the timed region.

Prints ONE JSON line.  value = densities carried through build + derivative
per second (nd / step time).  Also reported: builds/s and VJPs/s timed
separately, the mixed-precision build rate and its error when available,
per-kernel times from HIP events recorded around every launch during the
timed steps, the roofline fraction of the dominant kernel, sampled errors
against the CPU oracle, and the CPU oracle's own rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
PEAK_BF16_TFLOPS = 2516.6    # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E


# Kernel sources whose HBM traffic was measured with counters (the record in
# profiles/ names their sha256; a changed source voids the record).
TRAFFIC_SOURCES = {"half_transform": ["f64_core.hpp", "f64_mfma16.hpp", "jk_fp64.hip", "jk_tiles.hpp"]}


def measured_traffic(kernel, plan):
    """Bytes per launch (fetched + written) from the committed counter record
    taken under the same plan, or None when there is none for this kernel and
    plan or its sources changed since."""
    import glob
    import hashlib
    if kernel not in TRAFFIC_SOURCES:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2608_06536_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if line.startswith("traffic-record:"):
                rec = json.loads(line.split(":", 1)[1])
                if (rec.get("kernel") == kernel and rec.get("sources_sha256") == h.hexdigest()
                        and rec.get("plan") == [plan["ht_tile"], plan["chunk_mb"]]):
                    return rec["fetch_bytes"] + rec["write_bytes"]
    return None


# Derivative launches that run concurrently on two streams (stage B's two
# products): their HIP-event times include the concurrent launch.
OVERLAPPED = {"vjp_stage_b_p", "vjp_stage_b_r"}
# Launch names of one kernel function: the derivative's half-transforms are
# the build's kernel on chunks of their own.
SAME_KERNEL = {"vjp_half_transform": "half_transform"}


def kernel_models(p, nd, nao, naux, R):
    """Algorithmic work of each kernel over ONE step: (bound, amount, unit).
    Flops count the method's own products; bytes count one read of B's upper
    triangles for the HBM streams (gamma, omega, J), which need no more."""
    n2 = float(nao) * nao
    return {
        "half_transform": ("mfma", 4.0 * naux * n2 * R, "flop"),       # the build's
        "vjp_half_transform": ("mfma", 4.0 * naux * n2 * R, "flop"),   # the derivative's
        "exchange": ("mfma", 2.0 * naux * n2 * R, "flop"),
        "vjp_stage_b_p": ("mfma", 2.0 * naux * n2 * R, "flop"),
        "vjp_stage_b_r": ("mfma", 2.0 * naux * n2 * R, "flop"),
        "vjp_stage_c": ("mfma", 4.0 * naux * n2 * R, "flop"),
        "vjp_stage_d": ("mfma", 4.0 * naux * n2 * R, "flop"),
        "coulomb": ("hbm", 8.0 * naux * nao * (nao + 1) / 2, "byte"),   # B's upper triangles
        "project": ("hbm", 8.0 * naux * nao * (nao + 1) / 2, "byte"),   # gamma (build)
        "project16": ("hbm", 8.0 * naux * nao * (nao + 1) / 2, "byte"), # omega, gamma (derivative)
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision build")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate plans instead of loading the committed plan table")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-geometry batched leg")
    ap.add_argument("--plan", default="",
                    help="TILE,CHUNK_MB: use this plan instead of autotuning (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after the JSON line, run a plain copy kernel of known size "
                         "(read and write 1 GiB each) for HBM counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library runs one process on one GPU; sharding over GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_06536_amd import _lib, jk, synth

    p = synth.config(4)
    nd, nao, naux, r = p.nd, p.nao, p.naux, p.r
    R = nd * r
    t0 = time.time()
    B, CL, CR = synth.make_problem(p)
    W, V = synth.make_cotangents(p)
    print(f"# inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    Bd, Ld, Rd, Wd, Vd = (torch.from_numpy(a).to(dev) for a in (B, CL, CR, W, V))
    J = torch.empty((nd, nao, nao), dtype=torch.float64, device=dev)
    K = torch.empty_like(J)
    dB = torch.empty_like(Bd)
    dCL = torch.empty_like(Ld)
    dCR = torch.empty_like(Rd)
    nbytes = jk.workspace_bytes(jk.make_problem(nao, naux, nd, r))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    # plan of this shape: from the autotuner (untimed; jk_tune.h), or given
    # (the committed table by default, so that every run times the same plan)
    t_tune = time.perf_counter()
    plan_src = "paper_2608_06536_amd/tuned_plans.json"
    if args.plan:
        tile, mb = (int(v) for v in args.plan.split(","))
        jk.tuning_set(jk.make_problem(nao, naux, nd, r), tile, mb)
        plan_src = "--plan"
    elif args.autotune:
        jk.autotune(Bd, Ld, Rd, reps=5, out=(J, K), ws=ws)
        plan_src = "autotuned on this device"
    else:
        with open(os.path.join(ROOT, plan_src)) as fh:
            jk.tuning_load(fh.read())
    plan_fp64 = jk.tuning_get(jk.make_problem(nao, naux, nd, r))
    t_tune = time.perf_counter() - t_tune

    def build():
        jk.jk_build(Bd, Ld, Rd, out=(J, K), ws=ws)

    def vjp():
        jk.jk_vjp(Bd, Ld, Rd, Wd, Vd, out=(dB, dCL, dCR), ws=ws)

    def step():
        build()
        vjp()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps with every kernel launch bracketed by events
    _lib.prof_enable(4096)
    _lib.prof_reset()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    kern = _lib.prof_collect()
    dropped = _lib.prof_dropped()
    _lib.prof_disable()
    ms_per_step = 1e3 * t_total / args.steps
    value = nd * args.steps / t_total

    # ---- separate rates of the build and the derivative: median over n calls,
    # each bracketed by events on the calling stream (the library joins any
    # second stream back into it before returning)
    def rate(fn, n=20):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3

    t_build = rate(build)
    t_vjp = rate(vjp)

    # ---- mixed-precision build (INT8 slice products; gamma, J and all sums FP64)
    Jm = torch.empty_like(J)
    Km = torch.empty_like(K)
    mixed = {"mixed": "skipped"}
    try:
        if args.no_mixed:
            raise StopIteration
        nbm = jk.workspace_bytes(jk.make_problem(nao, naux, nd, r, "mixed"))
        wsm = torch.empty(nbm, dtype=torch.uint8, device=dev)

        def build_mixed():
            jk.jk_build(Bd, Ld, Rd, precision="mixed", out=(Jm, Km), ws=wsm)

        t_mixed = rate(build_mixed)
        build()
        torch.cuda.synchronize()
        errs = [float((Km[k] - K[k]).abs().max() / K[k].abs().max()) for k in range(nd)]
        mixed = {"builds_per_s_mixed": round(nd / t_mixed, 2), "build_ms_mixed": round(1e3 * t_mixed, 3),
                 "speedup_mixed_vs_fp64_build": round(t_build / t_mixed, 3),
                 "max_err_K_mixed_vs_fp64": max(errs),
                 "J_mixed_equals_fp64": bool(torch.equal(Jm, J))}
        # B's digit planes made once (jk_slice_b, timed on its own) and reused
        # by every build over the same B, as the paper's repeated builds on
        # fixed Cholesky vectors would (Sec. 2.1, 2.2)
        S = jk.slice_b(Bd, nao)
        t_slice = rate(lambda: jk.slice_b(Bd, nao, out=S), n=5)
        Kp = torch.empty_like(K)

        def build_mixed_pre():
            jk.jk_build(Bd, Ld, Rd, precision="mixed", out=(Jm, Kp), ws=wsm, slices=S)

        t_pre = rate(build_mixed_pre)
        torch.cuda.synchronize()
        mixed.update({"build_ms_mixed_presliced": round(1e3 * t_pre, 3),
                      "builds_per_s_mixed_presliced": round(nd / t_pre, 2),
                      "speedup_mixed_presliced_vs_fp64_build": round(t_build / t_pre, 3),
                      "slice_b_ms": round(1e3 * t_slice, 3), "slices_bytes": int(S.numel()),
                      "presliced_K_equals_mixed": bool(torch.equal(Kp, Km))})
        del wsm, S
    except StopIteration:
        pass
    except _lib.JKError as e:
        mixed = {"mixed": f"unavailable: {e}"}

    # ---- symmetric densities (the same factor for both sides: X-only path)
    try:
        Js = torch.empty_like(J)
        Ks = torch.empty_like(K)

        def build_sym():
            jk.jk_build(Bd, Ld, Ld, out=(Js, Ks), ws=ws)

        t_sym = rate(build_sym)

        def vjp_sym():
            jk.jk_vjp(Bd, Ld, Ld, Wd, Vd, out=(dB, dCL, dCR), ws=ws)

        t_vjp_sym = rate(vjp_sym)
        vjp()                      # the general adjoints again, for the sampled check below
        sym = {"builds_per_s_fp64_sym": round(nd / t_sym, 2), "build_ms_fp64_sym": round(1e3 * t_sym, 3),
               "speedup_vs_general_fp64": round(t_build / t_sym, 3),
               "vjp_ms_fp64_sym": round(1e3 * t_vjp_sym, 3),
               "vjp_speedup_vs_general_fp64": round(t_vjp / t_vjp_sym, 3)}
        if not args.no_mixed:
            wsm = torch.empty(jk.workspace_bytes(jk.make_problem(nao, naux, nd, r, "mixed")),
                              dtype=torch.uint8, device=dev)

            def build_sym_mixed():
                jk.jk_build(Bd, Ld, Ld, precision="mixed", out=(Js, Ks), ws=wsm)

            t_sym_m = rate(build_sym_mixed)
            sym.update({"builds_per_s_mixed_sym": round(nd / t_sym_m, 2),
                        "build_ms_mixed_sym": round(1e3 * t_sym_m, 3)})
            del wsm
        del Js, Ks
    except _lib.JKError as e:
        sym = {"symmetric": f"unavailable: {e}"}

    # ---- packed-triangular B (half the bytes of B in HBM)
    try:
        iu = torch.triu_indices(nao, nao, device=dev)
        Bpk = Bd[:, iu[0], iu[1]].contiguous()
        del iu
        Jp, Kp_ = torch.empty_like(J), torch.empty_like(K)
        packed = {"B_bytes": Bpk.numel() * 8}
        for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
            wsp = torch.empty(jk.workspace_bytes(jk.make_problem(nao, naux, nd, r, prec,
                                                                 packed=True)),
                              dtype=torch.uint8, device=dev)

            def build_packed():
                jk.jk_build(Bpk, Ld, Rd, precision=prec, out=(Jp, Kp_), ws=wsp)

            t_p = rate(build_packed)
            packed[f"build_ms_{prec}"] = round(1e3 * t_p, 3)
            packed[f"builds_per_s_{prec}"] = round(nd / t_p, 2)
            if prec == "fp64":
                # the derivative with packed B gives dB packed (half the bytes)
                dBpk = torch.empty_like(Bpk)

                def vjp_packed():
                    jk.jk_vjp(Bpk, Ld, Rd, Wd, Vd, out=(dBpk, dCL, dCR), ws=wsp)

                t_pv = rate(vjp_packed)
                packed["vjp_ms_fp64"] = round(1e3 * t_pv, 3)
                packed["vjps_per_s_fp64"] = round(nd / t_pv, 2)
                packed["vjp_workspace_bytes"] = int(wsp.numel())
                del dBpk
            del wsp
        del Bpk, Jp, Kp_
        vjp()                      # the general adjoints again, for the sampled check below
    except _lib.JKError as e:
        packed = {"packed": f"unavailable: {e}"}

    # ---- Fock combination 2J - a K - b K_lr in one call (second factor set:
    # a scaled copy of B in its own buffer, naux_lr = naux)
    try:
        Blr = Bd * 0.7
        Ff = torch.empty_like(J)
        fock = {"workload": "F = 2 J - 0.25 K - 0.75 K_lr, K_lr from a second set of "
                            f"{naux} Cholesky vectors, same densities"}
        for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
            wsf = torch.empty(int(_lib.lib().jk_fock_workspace_bytes(
                ctypes.byref(jk.make_problem(nao, naux, nd, r, prec)), naux)),
                dtype=torch.uint8, device=dev)

            def fock_call():
                jk.jk_fock(Bd, Ld, Rd, 2.0, -0.25, B_lr=Blr, c_lr=-0.75, precision=prec,
                           out=Ff, ws=wsf)

            t_f = rate(fock_call)
            fock[f"fock_ms_{prec}"] = round(1e3 * t_f, 3)
            fock[f"densities_per_s_{prec}"] = round(nd / t_f, 2)
            del wsf
        Jb, Kb = torch.empty_like(J), torch.empty_like(K)

        def separate():
            jk.jk_build(Bd, Ld, Rd, out=(J, K), ws=ws)
            jk.jk_build(Blr, Ld, Rd, want_j=False, out=(None, Kb), ws=ws)
            torch.add(2.0 * J, K, alpha=-0.25, out=Jb)
            Jb.add_(Kb, alpha=-0.75)

        t_sep = rate(separate)
        fock["separate_calls_ms_fp64"] = round(1e3 * t_sep, 3)
        del Blr, Ff, Jb, Kb
    except _lib.JKError as e:
        fock = {"fock": f"unavailable: {e}"}

    # ---- Laplace pseudo-density driver (same B; energy-scaled factors + J/K)
    try:
        from paper_2608_06536_amd import laplace as lap
        lo_, nvec_l, npts_l = synth.LAPLACE_BENCH
        Co, eo, Cv, ev, Xl = (torch.from_numpy(a).to(dev) for a in
                              (*synth.make_orbitals(lo_), synth.make_amplitudes(lo_, nvec_l)))
        t_r = time.perf_counter()
        x_lo, x_hi = lap.denominator_range(eo, ev)
        w_l, a_l, err_l, lev_l = lap.laplace_quadrature(npts_l, x_lo, x_hi)
        t_rule = time.perf_counter() - t_r
        nd_l = npts_l * nvec_l
        Jl = torch.empty((npts_l, nvec_l, nao, nao), dtype=torch.float64, device=dev)
        Kl = torch.empty_like(Jl)
        lap_res = {"workload": f"{npts_l} quadrature points x {nvec_l} amplitude matrix, "
                               f"nocc={lo_.nocc} nvir={lo_.nvir}: {nd_l} densities of rank "
                               f"{lo_.nocc}", "rule_points": npts_l, "rule_range": [x_lo, x_hi],
                   "rule_max_rel_err": err_l, "rule_is_minimax": lev_l,
                   "rule_host_s": round(t_rule, 3)}
        for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
            pl = lap.make_laplace_problem(nao, naux, lo_.nocc, lo_.nvir, nvec_l, npts_l, prec)
            wsl = torch.empty(int(_lib.lib().jk_laplace_workspace_bytes(ctypes.byref(pl))),
                              dtype=torch.uint8, device=dev)

            def build_lap():
                lap.laplace_jk(Bd, Co, eo, Cv, ev, Xl, rule=(w_l, a_l), precision=prec,
                               out=(Jl, Kl), ws=wsl)

            t_l = rate(build_lap)
            lap_res[f"densities_per_s_{prec}"] = round(nd_l / t_l, 2)
            lap_res[f"build_ms_{prec}"] = round(1e3 * t_l, 3)
            del wsl
        del Co, eo, Cv, ev, Xl, Jl, Kl
    except _lib.JKError as e:
        lap_res = {"laplace": f"unavailable: {e}"}

    # ---- the 64-geometry batch: nao uniform in [100, 500], naux = 4 nao, one
    # ground and five transition densities of rank nao / 10 (B totals 91 GB,
    # drawn on the device), one jk_build_batched call per precision, replayed
    # from its captured graph; beside it one jk_build per geometry
    batched = {"batched": "skipped"}
    if not args.no_batched:
        try:
            bprobs = synth.batched_problems()
            items = []
            for bp in bprobs:
                cl, cr = synth.make_factors(bp)
                items.append((synth.make_B_device(bp, dev), torch.from_numpy(cl).to(dev),
                              torch.from_numpy(cr).to(dev)))
            nd_tot = sum(bp.nd for bp in bprobs)
            bstream = torch.cuda.Stream()
            batched = {"workload": f"{len(bprobs)} geometries, nao uniform in [100, 500], naux = 4 nao, "
                                   "6 densities of rank nao/10 (1 ground + 5 transition); inputs drawn "
                                   "on the device", "densities": nd_tot,
                       "B_bytes": int(sum(8 * bp.naux * bp.nao ** 2 for bp in bprobs))}
            outs = [(torch.empty((bp.nd, bp.nao, bp.nao), dtype=torch.float64, device=dev),
                     torch.empty((bp.nd, bp.nao, bp.nao), dtype=torch.float64, device=dev))
                    for bp in bprobs]
            for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
                nbb = jk.batched_workspace_bytes([jk.make_problem(bp.nao, bp.naux, bp.nd, bp.r, prec)
                                                  for bp in bprobs])
                wsb = torch.empty(nbb, dtype=torch.uint8, device=dev)
                torch.cuda.synchronize()
                with torch.cuda.stream(bstream):
                    t_b = rate(lambda: jk.jk_build_batched(items, precision=prec, outs=outs, ws=wsb),
                               n=5)
                batched[f"batch_ms_{prec}"] = round(1e3 * t_b, 2)
                batched[f"densities_per_s_{prec}"] = round(nd_tot / t_b, 1)
                del wsb
                torch.cuda.empty_cache()
            wsg = torch.empty(max(jk.workspace_bytes(jk.make_problem(bp.nao, bp.naux, bp.nd, bp.r))
                                  for bp in bprobs), dtype=torch.uint8, device=dev)

            def singles():
                for (Bg, Lg, Rg), og in zip(items, outs):
                    jk.jk_build(Bg, Lg, Rg, out=og, ws=wsg)

            t_s = rate(singles, n=3)
            batched["one_build_per_geometry_ms_fp64"] = round(1e3 * t_s, 2)
            if "batch_ms_mixed" in batched:
                batched["speedup_mixed_batch_vs_fp64_batch"] = round(
                    batched["batch_ms_fp64"] / batched["batch_ms_mixed"], 3)
            del wsg
            # the same batch with every B packed (each full square freed as
            # its packed copy is made)
            for g in range(len(items)):
                Bg, Lg, Rg = items[g]
                iu = torch.triu_indices(Bg.shape[1], Bg.shape[1], device=dev)
                items[g] = (Bg[:, iu[0], iu[1]].contiguous(), Lg, Rg)
                del Bg, iu
            torch.cuda.empty_cache()
            batched["B_bytes_packed"] = int(sum(it[0].numel() * 8 for it in items))
            for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
                nbb = jk.batched_workspace_bytes([jk.make_problem(bp.nao, bp.naux, bp.nd, bp.r, prec,
                                                                  packed=True) for bp in bprobs])
                wsb = torch.empty(nbb, dtype=torch.uint8, device=dev)
                torch.cuda.synchronize()
                with torch.cuda.stream(bstream):
                    t_b = rate(lambda: jk.jk_build_batched(items, precision=prec, outs=outs, ws=wsb),
                               n=5)
                batched[f"batch_ms_{prec}_packed"] = round(1e3 * t_b, 2)
                del wsb
                torch.cuda.empty_cache()
            del items, outs
            torch.cuda.empty_cache()
        except (_lib.JKError, torch.cuda.OutOfMemoryError) as e:
            batched = {"batched": f"unavailable: {e}"}

    # ---- measured matrix-core peaks (the microbenchmark of jk_prof.h)
    peaks = {"int8_pops_random": round(_lib.peak_mfma("int8", True) / 1e15, 3),
             "int8_pops_constant": round(_lib.peak_mfma("int8", False) / 1e15, 3),
             "fp64_tflops_random": round(_lib.peak_mfma("fp64", True) / 1e12, 2),
             "note": "INT8 in the slice engine's 13-product pattern; random = uniform bytes per lane"}

    # ---- a library DGEMM of the half-transform's shape, for comparison: one
    # chunk of the plan as one (nq nao) x nao by nao x 2R product (torch.matmul
    # in FP64, served by the ROCm BLAS libraries); the kernel also writes the
    # per-slab X/Y layout, the library product one plain matrix
    try:
        nqc = jk.plan_describe(jk.make_problem(nao, naux, nd, r))["chunk_slabs"]
        A2 = Bd[:nqc].reshape(nqc * nao, nao)
        C2 = torch.randn((nao, 2 * R), dtype=torch.float64, device=dev)
        O2 = torch.empty((nqc * nao, 2 * R), dtype=torch.float64, device=dev)
        t_g = rate(lambda: torch.matmul(A2, C2, out=O2))
        peaks["library_dgemm_half_transform_shape"] = {
            "shape": [nqc * nao, nao, 2 * R], "ms": round(1e3 * t_g, 3),
            "tflops": round(2.0 * nqc * nao * nao * 2 * R / t_g / 1e12, 2)}
        del A2, C2, O2
    except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
        peaks["library_dgemm_half_transform_shape"] = f"unavailable: {e}"

    # ---- INT8 roofline of the mixed build's dominant kernel (event times of
    # the presliced build; the aux stream's slicing runs beside it, so the
    # rate is a lower bound)
    roof_mixed = None
    if isinstance(mixed, dict) and "build_ms_mixed_presliced" in mixed:
        wsm = torch.empty(jk.workspace_bytes(jk.make_problem(nao, naux, nd, r, "mixed")),
                          dtype=torch.uint8, device=dev)
        S = jk.slice_b(Bd, nao)
        for _ in range(2):
            jk.jk_build(Bd, Ld, Rd, precision="mixed", out=(Jm, Km), ws=wsm, slices=S)
        torch.cuda.synchronize()
        _lib.prof_enable(4096)
        _lib.prof_reset()
        nrep = 10
        for _ in range(nrep):
            jk.jk_build(Bd, Ld, Rd, precision="mixed", out=(Jm, Km), ws=wsm, slices=S)
        kmix = _lib.prof_collect()
        _lib.prof_disable()
        ops = {"ht_mixed": 13 * 4.0 * naux * nao * nao * R, "ex_mixed": 13 * 2.0 * naux * nao * nao * R}
        roof_mixed = {}
        for kname, kops in ops.items():
            if kname in kmix:
                kms, kcnt = kmix[kname]
                ach = kops * nrep / (kms * 1e-3) / 1e15
                roof_mixed[kname] = {"achieved": round(ach, 3), "unit": "int8 POP/s (13 digit-pair products)",
                                     "peak_nominal": 5.0, "frac_nominal": round(ach / 5.0, 3),
                                     "peak_measured_random": peaks["int8_pops_random"],
                                     "frac_measured": round(ach / peaks["int8_pops_random"], 3),
                                     "avg_launch_us": round(1e3 * kms / kcnt, 1),
                                     "overlapped": True}
        del wsm, S

    # ---- roofline of the dominant kernel
    models = kernel_models(p, nd, nao, naux, R)
    per_kernel = {}
    for name, (ms, cnt) in kern.items():
        ent = {"total_ms": round(ms, 3), "launches": cnt, "avg_us": round(1e3 * ms / max(cnt, 1), 1)}
        if name in models:
            bound, amount, unit = models[name]
            tot = amount * args.steps
            if unit == "flop":
                ent["tflops"] = round(tot / (ms * 1e-3) / 1e12, 2)
            else:
                ent["gbs"] = round(tot / (ms * 1e-3) / 1e9, 1)
        if name in OVERLAPPED:
            ent["overlapped"] = True
        per_kernel[name] = ent
    # The roofline kernel: the kernel function with the most time among those
    # that never share the GPU with another launch (an overlapped launch's
    # event time includes the other launch's work); its build launches (one
    # fixed chunk plan, the one the counter records cover) give the figures.
    fn_ms = {}
    for name, (ms, _) in kern.items():
        if name not in OVERLAPPED:
            fn = SAME_KERNEL.get(name, name)
            fn_ms[fn] = fn_ms.get(fn, 0.0) + ms
    dom = max(fn_ms, key=fn_ms.get)
    bound, amount, unit = models.get(dom, ("mfma", float("nan"), "flop"))
    dom_ms, dom_cnt = kern[dom]
    if unit == "flop":
        achieved = amount * args.steps / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 3),
                "traffic": measured_traffic(dom, plan_fp64), "traffic_unit": "HBM bytes per launch (counters)",
                "flop_per_launch": amount * args.steps / dom_cnt,
                "avg_launch_us": round(1e3 * dom_ms / dom_cnt, 1)}
    else:
        achieved = amount * args.steps / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 3),
                "traffic": measured_traffic(dom, plan_fp64), "traffic_unit": "HBM bytes per launch (counters)",
                "byte_per_launch": amount * args.steps / dom_cnt,
                "avg_launch_us": round(1e3 * dom_ms / dom_cnt, 1)}

    # the batched target as a rate ratio: densities/s of the mixed batched
    # build (members of nao 100-500) over densities/s of the FP64 build at
    # nao=500 (different workloads, compared per density)
    if "densities_per_s_mixed" in batched:
        batched["mixed_batch_rate_vs_fp64_build_rate"] = round(
            batched["densities_per_s_mixed"] / (nd / t_build), 3)
    out = {
        "metric": "J/K builds/s + VJPs/s at nao=500 (FP64 vs mixed), max err vs FP64 oracle",
        "value": round(value, 3),
        "unit": "densities/s (FP64 build + VJP)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "differentiated CD J/K build: nao=500 naux=2000, 8 non-symmetric "
                               "densities of rank 40, N(0,1) cotangents; step = jk_build + jk_vjp",
                   "nao": nao, "naux": naux, "ndens": nd, "rank": r, "precision": "fp64"},
        "builds_per_s_fp64": round(nd / t_build, 2),
        "vjps_per_s_fp64": round(nd / t_vjp, 2),
        "build_ms_fp64": round(1e3 * t_build, 3),
        "vjp_ms_fp64": round(1e3 * t_vjp, 3),
        "plan": {"fp64": plan_fp64, "source": plan_src, "plan_s": round(t_tune, 2)},
        "mixed": mixed,
        "symmetric_densities": sym,
        "packed_b": packed,
        "fock": fock,
        "laplace": lap_res,
        "batched": batched,
        "roofline": roof,
        "roofline_mixed": roof_mixed,
        "peaks_measured": peaks,
        "kernels": per_kernel,
        "prof_dropped": dropped,
    }

    # ---- sampled errors against the CPU oracle (same launch configuration)
    if not args.no_check:
        import oracle
        torch.cuda.synchronize()
        Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
        rng = np.random.default_rng(2024)
        n = 8
        ks, ms_, ns_ = rng.integers(0, nd, n), rng.integers(0, nao, n), rng.integers(0, nao, n)
        Je, Ke = oracle.jk_entries(B, CL, CR, ks, ms_, ns_)
        qs, as_, bs_ = rng.integers(0, naux, n), rng.integers(0, nao, n), rng.integers(0, nao, n)
        dBe = oracle.db_entries(B, CL, CR, W, V, qs, as_, bs_)
        dBh = dB[qs, as_, bs_].cpu().numpy()
        out["max_err_sampled"] = {
            "J": float(np.max(np.abs(Jh[ks, ms_, ns_] - Je)) / np.max(np.abs(Jh))),
            "K": float(np.max(np.abs(Kh[ks, ms_, ns_] - Ke)) / np.max(np.abs(Kh))),
            "dB": float(np.max(np.abs(dBh - dBe)) / float(dB.abs().max())),
            "entries_each": n,
        }

    # ---- CPU oracle baseline on a bounded Q-sample
    if not args.no_cpu:
        import oracle
        nthr = oracle.num_threads()

        def cpu_time(ns):
            Bs = np.ascontiguousarray(B[:ns])
            a = time.perf_counter()
            oracle.jk_factored(Bs, CL, CR)
            tf = time.perf_counter() - a
            a = time.perf_counter()
            oracle.vjp_factored(Bs, CL, CR, W, V)
            return tf, time.perf_counter() - a

        tf1, tv1 = cpu_time(2)
        per_slab = (tf1 + tv1) / 2
        ns = int(max(2, min(naux, args.cpu_seconds / max(per_slab, 1e-6))))
        tf, tv = cpu_time(ns) if ns > 2 else (tf1, tv1)
        scale = naux / ns
        t_cpu = (tf + tv) * scale
        # the nao=300 workload (naux=1200, 4 densities of rank 30) in full,
        # median of 3 builds
        p2 = synth.config(2)
        B2, CL2, CR2 = synth.make_problem(p2)
        t2 = []
        for _ in range(3):
            a = time.perf_counter()
            oracle.jk_factored(B2, CL2, CR2)
            t2.append(time.perf_counter() - a)
        out["cpu_baseline"] = {
            "value": round(nd / t_cpu, 5), "unit": "densities/s (FP64 build + VJP)",
            "cores": nthr, "kind": "oracle",
            "sample": f"factored oracle (build + derivative) on the first {ns} of {naux} slabs of "
                      f"the same workload, time scaled by {scale:.1f}",
            "build_s_est": round(tf * scale, 2), "vjp_s_est": round(tv * scale, 2),
            "nao300_build_s_median_of_3": round(float(np.median(t2)), 3),
            "nao300_densities_per_s": round(p2.nd / float(np.median(t2)), 4),
        }
    print(json.dumps(out), flush=True)

    if args.copy_calib:
        # y = x * 1 over 2^27 doubles: 1 GiB read + 1 GiB written per launch
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(f"# copy calibration: 3 launches, {x.numel() * 8} bytes read and written each",
              file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
