#!/usr/bin/env python3
"""Benchmark of the Brillouin-kernel overlap hot path on one MI355X.

Step (the timed unit behind `value`) = one pass of the whole hot path over one
synthetic batch: bri_build_links (U -> FP64 off-axis links) + ov_apply (FP64
multi-shift CG for the Kenney-Laub [16/16] rational, two stencil applies per
iteration, final apply) on a 16^4 lattice with smeared links (exp(0.5 i A),
3 APE steps at alpha 0.6), one normalised Gaussian source, rho = 1, CG
tolerance 1e-12 per shift.  This is the plain FP64 single-RHS GPU path.

value        overlap applies (right-hand sides) per second of that step
roofline     dominant kernel, the FP64 stencil bri_apply, timed live with HIP
             events on the library's stream: algorithmic bytes per launch
             (6144 B/site: the 40 stored links, spinor in and out) / average
             launch time, against the 8 TB/s HBM peak; `traffic` from the
             committed rocprofv3 counter summary when the kernel sources match
cpu_baseline the FP64 CPU oracle on a bounded sample (see `sample`)
extra        the same apply batched over the 12 spin-colour point sources and
             with mixed precision (FP32 / bfloat16-link inner solve, FP64
             refinement), each with its error against the FP64 result

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
       python bench.py --stencil-only     (copy calibration + stencil launches, for counters)
       python bench.py --stencil-only --lattice 32,32,32,64   (the same on a larger workload lattice)
       python bench.py --stencil-only --stencil-rhs 12        (plus the multi-RHS kernel, FP64 and FP32)
       python bench.py --batched-only --steps 5 --warmup 1    (12-source FP64 apply only, for traces)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
L_BENCH = (16, 16, 16, 16)
KL_N = 16
RHO = 1.0
CG_TOL = 1e-12
MASS = 0.05  # bare quark mass of the massive solve measured beside the apply
OUTER_TOL = 1e-10  # BiCGstab stop of that solve
LINK_EPS, APE_ALPHA, APE_STEPS = 0.5, 0.6, 3
LINK_SEED = 1701 + 2
SRC_SEED = 726 + 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_f64_16x16x16x16_counters.txt")


def stencil_bytes_per_site(spinor_bytes_per_real: int, link_bytes_per_real: int, nrhs: int = 1) -> int:
    """Algorithmic bytes of one stencil apply per site: 24 reals in and 24 out per
    right-hand side, and the 40 stored 3x3 complex links (720 reals)."""
    return (24 + 24) * nrhs * spinor_bytes_per_real + 720 * link_bytes_per_real


STENCIL_SOURCES = ("common.hpp", "stencil.hpp", "stencil_core.hpp", "stencil_kernels.hpp", "stencil.hip",
                   "stencil_f64_bri.hip", "tune.hip")


def kernel_source_digest() -> str:
    """Hash of the sources that define the FP64 stencil kernel and its launch configuration."""
    h = hashlib.sha256()
    for name in STENCIL_SOURCES:
        with open(os.path.join(ROOT, "paper_1701_00726_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the FP64 stencil at 16^4 from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its copy-kernel factor), or
    None when the kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for ln in f:
            if "=" in ln and not ln.startswith("#"):
                k, v = ln.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_src_sha") != kernel_source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--stencil-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and mixed-precision measurements")
    ap.add_argument("--tune", action="store_true", help="autotune the stencil launch before timing")
    ap.add_argument("--survey", action="store_true",
                    help="stencil (tuned, FP64/FP32/BF16-link, 1 and 12 RHS) and overlap timings at 16^4, 24^3x48, 32^3x64")
    ap.add_argument("--stencil-only", action="store_true", help="copy calibration + stencil launches only")
    ap.add_argument("--stencil-rhs", type=int, default=1,
                    help="with --stencil-only: also launch the multi-RHS kernel on this many RHS (FP64 and FP32)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 12-source FP64 overlap apply, --steps times (for kernel traces)")
    ap.add_argument("--lattice", default=None,
                    help="with --stencil-only: another lattice, e.g. 32,32,32,64 (links exp(0.7iA) + 3 APE "
                         "built on the device)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    return ap.parse_args()


def cpu_baseline(L, U_np, shift_iters, budget_s):
    """Time the FP64 oracle on a bounded sample of the same workload and scale it
    to one overlap apply: oracle links + sum over shifts of (per-shift CG iterations
    x measured time per CG iteration) + the final stencil apply."""
    import oracle
    import synth
    from oracle import kl

    t0 = time.perf_counter()
    Wo = oracle.links(L, U_np)
    t_links = time.perf_counter() - t0
    b = synth.gaussian_source(L, SRC_SEED)[0]
    _, _, sg = kl.kl_diag_coeffs_f64(KL_N)
    its = 2
    while True:
        t0 = time.perf_counter()
        oracle.cg(L, Wo, -RHO, sg[0], b, tol=1e-30, maxit=its)
        dt = time.perf_counter() - t0
        # one restart residual + `its` iterations + the final true residual = its + 2 normal-op applies
        t_iter = dt / (its + 2)
        if dt * 2.5 > budget_s or its >= 64:
            break
        its *= 2
    t0 = time.perf_counter()
    oracle.dirac(L, Wo, -RHO, b)
    t_apply = time.perf_counter() - t0
    total_iters = int(sum(shift_iters))
    t_est = t_links + total_iters * t_iter + t_apply
    return {
        "value": 1.0 / t_est,
        "unit": "overlap applies/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (
            f"oracle links ({t_links:.2f} s) + {its} CG iterations of the smallest shift "
            f"({t_iter:.3f} s each) + one stencil apply ({t_apply:.2f} s) timed on {L[0]}x{L[1]}x{L[2]}x{L[3]}; "
            f"scaled to the {total_iters} per-shift CG iterations ({KL_N} shifts solved one by one) "
            f"that one apply needs: {t_est:.1f} s per apply"
        ),
    }


def survey(torch, bri, synth):
    """Tuned stencil and overlap timings at the three workload lattices (links
    exp(i eps A) + 3 APE(0.6) built on the device; one JSON line per lattice)."""
    cfgs = [((16, 16, 16, 16), 0.5, 1703), ((24, 24, 24, 48), 0.7, 1704), ((32, 32, 32, 64), 0.7, 1705)]
    name = {bri.F64: "f64", bri.F32: "f32", bri.F32_BF16W: "bf16w"}
    bps = {bri.F64: 8, bri.F32: 4, bri.F32_BF16W: 4}
    bpl = {bri.F64: 8, bri.F32: 4, bri.F32_BF16W: 2}
    for L, eps, seed in cfgs:
        V = int(np.prod(L))
        U = synth.smeared_links_torch(L, eps, seed, APE_ALPHA, APE_STEPS, device="cuda", chunk=1 << 18)
        U = U.permute(0, 2, 3, 1).contiguous()
        W = {p: bri.build_links(L, U, p) for p in (bri.F64, bri.F32, bri.F32_BF16W)}
        del U
        rec = {"lattice": list(L), "link_eps": eps}
        g = torch.randn((12, 4, 3, V), dtype=torch.complex128, device="cuda")
        for p in (bri.F64, bri.F32, bri.F32_BF16W):
            for nr in (1, 12):
                x = g[:nr].to(bri.spinor_dtype(p)).contiguous()
                best, us = bri.autotune(L, W[p], p, x, reps=3)
                key = f"stencil_{name[p]}_{nr}rhs"
                rec[key] = {"us": us, "GBps_alg": stencil_bytes_per_site(bps[p], bpl[p], nr) * V / us / 1e3,
                            "config": best.as_dict()}
                print(f"[survey] {L} {key} {us:.1f} us", file=sys.stderr, flush=True)
        b1 = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED), bri.F64)
        b12 = bri.spinor_to_device(synth.point_sources_12(L), bri.F64)
        # the last row keeps every (shift, source) solution in FP64 for the refinement: 16 x 12 columns,
        # 77 GB at 32^3x64, ~210 GB of HBM with the FP32 multi-shift and the link arrays
        for nm, inner, b in (("fp64_1src", bri.F64, b1), ("fp64_12src", bri.F64, b12), ("mixed_f32_1src", bri.F32, b1),
                             ("mixed_f32_12src", bri.F32, b12)):
            op = bri.OverlapOp(L, W[bri.F64], kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000,
                               Wlo=None if inner == bri.F64 else W[inner], inner=inner, nrhs=b.shape[0])
            op.apply(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = op.apply(b)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec["overlap_" + nm] = {"ms_per_call": dt * 1e3, "applies_per_s": b.shape[0] / dt, "cg_iters": st.iters,
                                    "refine_passes": st.refine}
            print(f"[survey] {L} overlap {nm} {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
            del op
            torch.cuda.empty_cache()
        print(json.dumps(rec), flush=True)
        del W, g
        torch.cuda.empty_cache()


def stencil_only_large(torch, bri, synth, L, reps):
    """Counter runs on a workload lattice other than the bench's: a 1 GiB calibration copy, the
    links of that lattice's recipe (exp(0.7 i A) + 3 APE(0.6)) built on the device, and `reps`
    FP64 stencil launches in the default configuration."""
    V = int(np.prod(L))
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    del a, c
    U = synth.smeared_links_torch(L, 0.7, LINK_SEED, APE_ALPHA, APE_STEPS, device="cuda", chunk=1 << 18)
    W = bri.build_links(L, U.permute(0, 2, 3, 1).contiguous(), bri.F64)
    del U
    x = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED), bri.F64)
    y = torch.empty_like(x)
    for _ in range(reps):
        bri.apply(L, W, bri.F64, -RHO, x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"stencil_only": True, "lattice": list(L), "launches": reps,
                      "alg_bytes_per_launch": stencil_bytes_per_site(8, 8) * V,
                      "config": bri.get_stencil_cfg(L, bri.F64, 1).as_dict()}), flush=True)


# the cascaded-preconditioning measurement: the 16^3x32 volume of the paper's timing table,
# links exp(0.5 iA) + 7 APE(0.6) steps, am = 0.03, rho = 1, exit |r|/|b| <= 1e-9
CASCADE_L = (16, 16, 16, 32)
CASCADE_MASS, CASCADE_TOL, CASCADE_APE = 0.03, 1e-9, 7
# rows: (Kenney-Laub order, name, preconditioner levels as (kl_n, tol, max_iter, ms_tol, precision),
# sources side by side); the first four are the paper's table, then the preconditioners in FP32
# (their accuracy does not reach the result) and the 12-source batch
CASCADE_ROWS = (
    (1, "none", (), 1),
    (1, "1-level", ((0, 0.03, 50, 0.0, 0),), 1),
    (4, "none", (), 1),
    (4, "2-level", ((1, 0.03, 30, 1e-4, 0), (0, 0.1, 30, 0.0, 0)), 1),
    (1, "1-level, FP32 level", ((0, 0.03, 50, 0.0, 1),), 1),
    (4, "2-level, FP32 levels", ((1, 0.03, 30, 1e-4, 1), (0, 0.1, 30, 0.0, 1)), 1),
    (1, "1-level, FP32 level, 12 sources", ((0, 0.03, 50, 0.0, 1),), 12),
    (4, "2-level, FP32 kernel level, 12 sources", ((1, 0.03, 30, 1e-4, 0), (0, 0.1, 30, 0.0, 1)), 12),
)


# the operator-quality comparison of Sec. 7: the f_{1,1} overlap (rho = 1) with Brillouin or Wilson
# kernel, 1 or 3 APE steps (alpha = 0.72, the paper's), c_SW = 0 or 1, on a 16^3x32 field
QUALITY_L = (16, 16, 16, 32)
QUALITY_APE_ALPHA = 0.72


def quality_table(dev):
    """Normality and Ginsparg-Wilson defects (mean over 4 Gaussian vectors) and the locality decay
    rate delta (mean over 2 point sources) for each kernel setting."""
    import torch

    import paper_1701_00726_amd as bri
    import synth
    from paper_1701_00726_amd import quality

    L = QUALITY_L
    V = int(np.prod(L))
    rows = []
    eta = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED + 40, nrhs=4), bri.F64, dev)
    for ape in (1, 3):
        U = synth.smeared_links_torch(L, LINK_EPS, LINK_SEED + 40, QUALITY_APE_ALPHA, ape, device=dev, chunk=1 << 18)
        U = U.permute(0, 2, 3, 1).contiguous()
        for csw in (0.0, 1.0):
            W = bri.build_links(L, U, bri.F64, csw=csw)
            for kname, kernel in (("brillouin", bri.KERNEL_BRILLOUIN), ("wilson", bri.KERNEL_WILSON)):
                op = bri.OverlapOp(L, W, kl_n=1, rho=1.0, tol=1e-12, max_iter=20000, kernel=kernel, nrhs=4)
                t0 = time.perf_counter()
                nd = quality.normality_defect(op, eta)
                gw = quality.gw_defect(op, eta)
                deltas = []
                for seed in (1, 2):
                    r, mag = quality.locality_profile(op, L, quality.point_source(L, seed, dev))
                    deltas.append(quality.decay_rate(r, mag, rmin=2.0, rmax=8.0))
                torch.cuda.synchronize()
                rows.append({"kernel": kname, "ape_steps": ape, "csw": csw, "normality": float(np.mean(nd)),
                             "gw_defect": float(np.mean(gw)), "locality_delta": float(np.mean(deltas)),
                             "seconds": time.perf_counter() - t0})
                del op
            del W
        del U
    return {"lattice": list(L), "operator": "f_{1,1} overlap, rho = 1", "ape_alpha": QUALITY_APE_ALPHA,
            "rows": rows}


def cascade_table(dev):
    """Outer BiCGstab iterations and seconds per right-hand side for f_{1,1} and f_{4,4}, without
    and with cascaded preconditioning (complete massive form), one Gaussian source."""
    import torch

    import paper_1701_00726_amd as bri
    import synth

    L = CASCADE_L
    U = synth.smeared_links_torch(L, LINK_EPS, LINK_SEED + 30, APE_ALPHA, CASCADE_APE, device=dev, chunk=1 << 18)
    U = U.permute(0, 2, 3, 1).contiguous()
    W = bri.build_links(L, U, bri.F64)
    W32 = bri.build_links(L, U, bri.F32)
    del U
    b1 = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED + 30), bri.F64, dev)
    b12 = bri.spinor_to_device(synth.point_sources_12(L), bri.F64, dev)
    rows, ref = [], {}
    for n, name, levels, nsrc in CASCADE_ROWS:
        b = b1 if nsrc == 1 else b12
        prec = [bri.Level(k, tol=t, max_iter=mi, ms_tol=ms, inner=ip) for k, t, mi, ms, ip in levels]
        op = bri.OverlapOp(L, W, kl_n=n, rho=RHO, tol=CG_TOL, max_iter=5000, Wlo=W32)
        op.solve(b, CASCADE_MASS, tol=1e-3, prec=prec)  # warm caches and workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = op.solve(b, CASCADE_MASS, complete=True, tol=CASCADE_TOL, max_iter=2000, prec=prec)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / nsrc
        row = {"f": f"{n},{n}", "precond": name, "n_iter": st.iters, "s_per_rhs": sec, "sources": nsrc,
               "level_iters": st.level_iters, "true_rel_resid": st.rel_resid}
        key = (n, nsrc)
        if key in ref:
            row["rel_diff_vs_first_row"] = float(torch.linalg.vector_norm(x - ref[key]) /
                                                 torch.linalg.vector_norm(ref[key]))
        else:
            ref[key] = x
        rows.append(row)
        del op
    return {"lattice": list(L), "mass": CASCADE_MASS, "tol": CASCADE_TOL, "ape_steps": CASCADE_APE, "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(
            "bench.py measures one GPU only: the library has no multi-GPU path "
            "(the work would shard by sources, or by domain decomposition of the lattice in t).",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    import paper_1701_00726_amd as bri
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.survey:
        survey(torch, bri, synth)
        return
    if args.stencil_only and args.lattice:
        stencil_only_large(torch, bri, synth, tuple(int(v) for v in args.lattice.split(",")), args.stencil_reps)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    L = L_BENCH
    V = int(np.prod(L))

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps  # ms

    print(f"[bench] generating links {L} eps={LINK_EPS} APE {APE_STEPS}x{APE_ALPHA}", file=sys.stderr, flush=True)
    U_np = synth.smeared_links(L, LINK_EPS, LINK_SEED, APE_ALPHA, APE_STEPS)
    U = bri.links_to_device(U_np, dev)
    b = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED), bri.F64, dev)
    W = torch.empty((40, 3, 3, V), dtype=torch.complex128, device=dev)
    out = torch.empty_like(b)
    bri.build_links(L, U, bri.F64, out=W)
    if args.tune:
        cfg, us = bri.autotune(L, W, bri.F64, b, reps=5)
        print(f"[bench] tuned FP64 stencil: {us:.1f} us {cfg.as_dict()}", file=sys.stderr, flush=True)
    tuned = bri.get_stencil_cfg(L, bri.F64, 1).as_dict()

    if args.stencil_only:
        # calibration copy of 1 GiB (beyond the 256 MB Infinity Cache), then the stencil
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        t_in, t_out = b.clone(), torch.empty_like(b)
        for _ in range(args.stencil_reps):
            bri.apply(L, W, bri.F64, -RHO, t_in, out=t_out)
        torch.cuda.synchronize()
        rec = {"stencil_only": True, "launches": args.stencil_reps, "copy_bytes": 1 << 30,
               "kernel_src_sha": kernel_source_digest(), "config": tuned}
        if args.stencil_rhs > 1:
            # the multi-RHS kernel in its default configuration, FP64 and FP32 links and vectors
            nr = args.stencil_rhs
            src = synth.gaussian_source(L, SRC_SEED, nrhs=nr)
            for prec, name in ((bri.F64, "f64"), (bri.F32, "f32")):
                Wp = W if prec == bri.F64 else bri.build_links(L, U, prec)
                xm = bri.spinor_to_device(src, prec, dev)
                ym = torch.empty_like(xm)
                bri.apply(L, Wp, prec, -RHO, xm, out=ym)  # first launch loads the kernel's code object
                ms = timed(lambda: bri.apply(L, Wp, prec, -RHO, xm, out=ym), args.stencil_reps)
                rec[f"mrhs_{name}_{nr}rhs"] = {"us": ms * 1e3, "config": bri.get_stencil_cfg(L, prec, nr).as_dict()}
                del Wp, xm, ym
        print(json.dumps(rec), flush=True)
        return

    if args.batched_only:
        # the 12 spin-colour point sources side by side, one multi-shift with per-column scalars
        b12 = bri.spinor_to_device(synth.point_sources_12(L), bri.F64, dev)
        o12 = torch.empty_like(b12)
        op12 = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, nrhs=12)
        for _ in range(args.warmup):
            op12.apply(b12, out=o12)
        ms = timed(lambda: op12.apply(b12, out=o12), args.steps)
        _, st12 = op12.apply(b12, out=o12)
        print(json.dumps({"batched_only": True, "sources": 12, "calls": args.steps, "ms_per_call": ms,
                          "applies_per_s": 12 / (ms / 1e3), "cg_iterations": st12.iters,
                          "config": bri.get_stencil_cfg(L, bri.F64, 12).as_dict()}), flush=True)
        return

    op = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000)

    def step():
        bri.build_links(L, U, bri.F64, out=W)
        _, st = op.apply(b, out=out)
        return st

    for _ in range(args.warmup):
        st = step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done, {st.iters} CG iterations per apply", file=sys.stderr, flush=True)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    iters = []
    for _ in range(args.steps):
        st = step()
        iters.append(st.iters)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = b.shape[0] / (ms_step / 1e3)
    ref64 = out.clone()
    print(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step (host wall {wall:.3f} s)", file=sys.stderr, flush=True)

    # dominant kernel: the FP64 stencil, timed live with events on the same stream
    t_in, t_out = b.clone(), torch.empty_like(b)
    for _ in range(5):
        bri.apply(L, W, bri.F64, -RHO, t_in, out=t_out)
    torch.cuda.synchronize()
    ms_launch = timed(lambda: bri.apply(L, W, bri.F64, -RHO, t_in, out=t_out), args.stencil_reps)
    us_launch = ms_launch * 1e3
    alg_bytes = stencil_bytes_per_site(8, 8) * V
    achieved = alg_bytes / (us_launch * 1e-6) / 1e9
    traffic = measured_traffic()
    print(f"[bench] bri_apply FP64 {us_launch:.1f} us/launch, {achieved:.0f} GB/s", file=sys.stderr, flush=True)

    result = {
        "metric": "D_bri apply GB/s (% HBM peak); overlap applies/s at 1e-10, mixed vs FP64",
        "value": value,
        "unit": "overlap applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "16^4 FP64 single-RHS overlap apply, Kenney-Laub [16/16], rho=1, CG tol 1e-12, "
            "links exp(0.5iA) + 3 APE(0.6), Gaussian source; step = bri_build_links + ov_apply",
            "lattice": list(L),
            "kl_n": KL_N,
            "nrhs": int(b.shape[0]),
            "precision": "fp64",
            "cg_iterations": int(np.median(iters)),
            "stencil_config": tuned,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "bri_apply FP64 1-RHS (stencil_kernel<LinkF64,nsplit,false,EPI_PLAIN>)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None if traffic is None else traffic / (us_launch * 1e-6) / 1e9,
            "traffic_bytes_per_launch": traffic,
            "us_per_launch": us_launch,
            "alg_bytes_per_launch": alg_bytes,
        },
    }

    if not args.no_extra:
        extra = {}
        # 12 spin-colour point sources, batched FP64
        b12 = bri.spinor_to_device(synth.point_sources_12(L), bri.F64, dev)
        o12 = torch.empty_like(b12)
        if args.tune:
            bri.autotune(L, W, bri.F64, b12, reps=3)
        op12 = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, nrhs=12)
        op12.apply(b12, out=o12)
        ms = timed(lambda: op12.apply(b12, out=o12), 3)
        extra["batched_fp64_12src"] = {"applies_per_s": 12 / (ms / 1e3), "ms_per_call": ms}
        ref12 = o12.clone()
        # single-source FP64 on the point source 0 for the per-solve error of the mixed runs
        for name, inner in (("mixed_f32", bri.F32), ("mixed_bf16w", bri.F32_BF16W)):
            Wlo = bri.build_links(L, U, inner)
            opm = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, Wlo=Wlo, inner=inner)
            om = torch.empty_like(b)
            _, stm = opm.apply(b, out=om)
            ms = timed(lambda: opm.apply(b, out=om), 2)
            err = float(torch.linalg.vector_norm(om - ref64) / torch.linalg.vector_norm(ref64))
            extra[name + "_1src"] = {"applies_per_s": 1 / (ms / 1e3), "ms_per_call": ms, "refine_passes": stm.refine,
                                     "rel_err_vs_fp64": err}
            opm12 = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, Wlo=Wlo, inner=inner, nrhs=12)
            om12 = torch.empty_like(b12)
            opm12.apply(b12, out=om12)
            ms = timed(lambda: opm12.apply(b12, out=om12), 1)
            errs = [float(torch.linalg.vector_norm(om12[r] - ref12[r]) / torch.linalg.vector_norm(ref12[r]))
                    for r in range(12)]
            extra[name + "_12src"] = {"applies_per_s": 12 / (ms / 1e3), "ms_per_call": ms,
                                      "max_rel_err_vs_fp64": max(errs)}
            del opm, opm12, Wlo
            torch.cuda.empty_cache()
        # HIP-graph replay of the CG loop against plain launches, here and on a small lattice
        graphs = {}
        for Lg in (L, (8, 8, 8, 8)):
            if Lg == L:
                opg, bg = op, b
            else:
                Ug = bri.links_to_device(synth.smeared_links(Lg, LINK_EPS, LINK_SEED, APE_ALPHA, APE_STEPS), dev)
                Wg = bri.build_links(Lg, Ug, bri.F64)
                opg = bri.OverlapOp(Lg, Wg, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000)
                bg = bri.spinor_to_device(synth.gaussian_source(Lg, SRC_SEED), bri.F64, dev)
            og = torch.empty_like(bg)
            row = {}
            for on in (False, True):
                bri.set_solver_graphs(on)
                opg.apply(bg, out=og)
                row["ms_graphs_on" if on else "ms_graphs_off"] = timed(lambda: opg.apply(bg, out=og), 10)
            graphs["x".join(str(v) for v in Lg)] = row
        extra["cg_graph_replay"] = graphs
        # gradient of Re chi^dag D_ov psi (force on the links and D_ov^dag chi), FP64
        chi = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED + 1), bri.F64, dev)
        op.grad(U, chi[0], b[0])
        ms_g = timed(lambda: op.grad(U, chi[0], b[0]), 2)
        pairs = [(1.0, chi[0], b[0])] * (2 * KL_N + 1)
        bri.link_grad(L, U, W, pairs)
        ms_f = timed(lambda: bri.link_grad(L, U, W, pairs), 3)
        extra["grad_fp64_1src"] = {"ms_per_call": ms_g, "ratio_to_step": ms_g / ms_step,
                                   "link_force_ms_%d_pairs" % (2 * KL_N + 1): ms_f}
        # the Wilson kernel (eq. (def_wils)) on the same links: its 9-point stencil (four link
        # matrices, one spinor in and out per site: 960 B/site in FP64) and its overlap apply
        for _ in range(5):
            bri.wilson_apply(L, W, bri.F64, -RHO, t_in, out=t_out)
        ms_w = timed(lambda: bri.wilson_apply(L, W, bri.F64, -RHO, t_in, out=t_out), args.stencil_reps)
        opw = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=20000, kernel=bri.KERNEL_WILSON)
        ow = torch.empty_like(b)
        _, stw = opw.apply(b, out=ow)
        ms_ow = timed(lambda: opw.apply(b, out=ow), 3)
        extra["wilson_kernel_fp64_1src"] = {
            "stencil_us": ms_w * 1e3, "stencil_GBps_alg": 960 * V / (ms_w * 1e-3) / 1e9,
            "overlap_applies_per_s": 1 / (ms_ow / 1e3), "overlap_ms_per_call": ms_ow, "cg_iterations": stw.iters,
            "brillouin_cg_iterations": int(np.median(iters)), "brillouin_stencil_us": us_launch}
        del opw, ow
        # relaxed per-shift stopping (tol * omega_max / omega_i) against the strict apply
        opr = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, relax=True)
        orl = torch.empty_like(b)
        _, str_ = opr.apply(b, out=orl)
        ms_r = timed(lambda: opr.apply(b, out=orl), 10)
        extra["relaxed_fp64_1src"] = {
            "applies_per_s": 1 / (ms_r / 1e3), "ms_per_call": ms_r, "cg_iterations": str_.iters,
            "rel_diff_vs_strict": float(torch.linalg.vector_norm(orl - ref64) / torch.linalg.vector_norm(ref64))}
        del opr, orl
        # the first upper-diagonal rational g_{2n} (Sec. 3.3; no constant term), n = KL_N shifts
        opu = bri.OverlapOp(L, W, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000, kind=bri.KL_UPPER)
        ou = torch.empty_like(b)
        _, stu = opu.apply(b, out=ou)
        ms_u = timed(lambda: opu.apply(b, out=ou), 10)
        extra["upper_diagonal_fp64_1src"] = {
            "applies_per_s": 1 / (ms_u / 1e3), "ms_per_call": ms_u, "cg_iterations": stu.iters,
            "rel_diff_vs_diagonal": float(torch.linalg.vector_norm(ou - ref64) / torch.linalg.vector_norm(ref64))}
        del opu, ou
        # the clover-improved Brillouin kernel, c_SW = 1: 72 clover entries per site after the 40
        # link slabs (7296 B/site algorithmic in FP64), and its overlap apply
        Wc = bri.build_links(L, U, bri.F64, csw=1.0)
        for _ in range(5):
            bri.apply(L, Wc, bri.F64, -RHO, t_in, out=t_out)
        ms_c = timed(lambda: bri.apply(L, Wc, bri.F64, -RHO, t_in, out=t_out), args.stencil_reps)
        opc = bri.OverlapOp(L, Wc, kl_n=KL_N, rho=RHO, tol=CG_TOL, max_iter=5000)
        oc = torch.empty_like(b)
        _, stc = opc.apply(b, out=oc)
        ms_oc = timed(lambda: opc.apply(b, out=oc), 10)
        extra["clover_fp64_1src"] = {
            "csw": 1.0, "stencil_us": ms_c * 1e3, "stencil_GBps_alg": 7296 * V / (ms_c * 1e-3) / 1e9,
            "overlap_applies_per_s": 1 / (ms_oc / 1e3), "overlap_ms_per_call": ms_oc, "cg_iterations": stc.iters}
        del Wc, opc, oc
        # massive overlap solve, complete form of Sec. 4 with the BiCGstab outer solver, am = 0.05
        xs, sts = op.solve(b, MASS, complete=True, tol=OUTER_TOL)
        ms_s = timed(lambda: op.solve(b, MASS, complete=True, tol=OUTER_TOL), 1)
        extra["massive_solve_fp64_1src"] = {
            "mass": MASS, "outer_tol": OUTER_TOL, "outer_iters": sts.iters, "ov_applies": sts.applies,
            "inner_cg_iters": sts.inner_iters, "ms_per_solve": ms_s, "ms_per_ov_apply": ms_s / sts.applies,
            "true_rel_resid": sts.rel_resid}
        del xs
        # the same solve for the 12 spin-colour point sources side by side (the paper's batch)
        x12, st12 = op12.solve(b12, MASS, complete=True, tol=OUTER_TOL)
        ms_s12 = timed(lambda: op12.solve(b12, MASS, complete=True, tol=OUTER_TOL), 1)
        extra["massive_solve_fp64_12src"] = {
            "mass": MASS, "outer_tol": OUTER_TOL, "outer_iters": st12.iters, "ms_per_solve": ms_s12,
            "ms_per_rhs": ms_s12 / 12, "speedup_per_rhs_vs_1src": ms_s / (ms_s12 / 12),
            "true_rel_resid_worst": st12.rel_resid}
        del x12
        extra["cascaded_16x16x16x32"] = cascade_table(dev)
        extra["kernel_quality_16x16x16x32"] = quality_table(dev)
        best_mixed = max(extra[k]["applies_per_s"] for k in extra if k.startswith("mixed"))
        extra["fp64_1src_applies_per_s"] = value
        extra["speedup_batched_fp64_vs_fp64_1src"] = extra["batched_fp64_12src"]["applies_per_s"] / value
        extra["speedup_best_mixed_vs_fp64_1src"] = best_mixed / value
        result["extra"] = extra
        print(f"[bench] extra: {json.dumps(extra)}", file=sys.stderr, flush=True)

    if not args.no_cpu:
        print("[bench] CPU oracle sample ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(L, U_np, st.shift_iters, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
