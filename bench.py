#!/usr/bin/env python3
"""Benchmark of the Brillouin-kernel overlap hot path on one MI355X.

Step = one pass of the whole hot path over one synthetic batch:
  bri_build_links (U -> FP64 off-axis links) + ov_apply (multi-shift CG for the
  Kenney-Laub [16/16] rational, 2 stencil applies per iteration, final apply)
on a 16^4 lattice with smeared links (exp(0.5 i A), 3 APE steps at alpha 0.6)
and one normalised Gaussian source, FP64, rho = 1, CG tolerance 1e-12.

value      = overlap applies (right-hand sides) per second over the timed steps
roofline   = the dominant kernel, the FP64 stencil bri_apply, timed live with
             HIP events on the library's stream: algorithmic bytes per launch
             (6144 B/site: 40 stored links + spinor in + spinor out) / average
             launch time, against the 8 TB/s HBM peak
cpu_baseline = the FP64 CPU oracle on a bounded sample (see `sample`)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

from __future__ import annotations

import argparse
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
LINK_EPS, APE_ALPHA, APE_STEPS = 0.5, 0.6, 3
LINK_SEED = 1701 + 2
SRC_SEED = 726 + 2


def stencil_bytes_per_site(spinor_bytes_per_real: int, link_bytes_per_real: int, nrhs: int = 1) -> int:
    """Algorithmic bytes of one stencil apply per site: 24 reals in and 24 out per
    right-hand side, and the 40 stored 3x3 complex links (720 reals)."""
    return (24 + 24) * nrhs * spinor_bytes_per_real + 720 * link_bytes_per_real


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--stencil-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    return ap.parse_args()


def cpu_baseline(L, U_np, shift_iters, budget_s):
    """Time the FP64 oracle on a bounded sample of the same workload and scale it
    to one overlap apply: oracle links + sum over shifts of (per-shift CG iterations
    x measured time per CG iteration) + the final stencil apply."""
    import oracle

    t0 = time.perf_counter()
    Wo = oracle.links(L, U_np)
    t_links = time.perf_counter() - t0
    b = __import__("synth").gaussian_source(L, SRC_SEED)[0]
    c0, om, sg = __import__("oracle.kl", fromlist=["kl"]).kl_diag_coeffs_f64(KL_N)
    # CG iterations on the smallest shift until the budget is used (at least 2)
    t_iter = None
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


def main():
    args = parse()
    if args.gpus != 1:
        print(
            "bench.py measures one GPU only: this build has no multi-GPU path "
            "(the lattice would shard by sources or by domain decomposition; see the design notes).",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    import paper_1701_00726_amd as bri
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    L = L_BENCH
    V = int(np.prod(L))

    print(f"[bench] generating links {L} eps={LINK_EPS} APE {APE_STEPS}x{APE_ALPHA}", file=sys.stderr, flush=True)
    U_np = synth.smeared_links(L, LINK_EPS, LINK_SEED, APE_ALPHA, APE_STEPS)
    U = bri.links_to_device(U_np, dev)
    b = bri.spinor_to_device(synth.gaussian_source(L, SRC_SEED), bri.F64, dev)
    W = torch.empty((40, 3, 3, V), dtype=torch.complex128, device=dev)
    out = torch.empty_like(b)
    bri.build_links(L, U, bri.F64, out=W)
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
    value = args.steps * b.shape[0] / (ms_step * args.steps / 1e3)
    print(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step (host wall {wall:.3f} s)", file=sys.stderr, flush=True)

    # dominant kernel: the FP64 stencil, timed live with events on the same stream
    t_in = torch.empty_like(b)
    t_out = torch.empty_like(b)
    t_in.copy_(b)
    for _ in range(5):
        bri.apply(L, W, bri.F64, -RHO, t_in, out=t_out)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.stencil_reps):
        bri.apply(L, W, bri.F64, -RHO, t_in, out=t_out)
    s1.record(stream)
    torch.cuda.synchronize()
    us_launch = s0.elapsed_time(s1) * 1e3 / args.stencil_reps
    alg_bytes = stencil_bytes_per_site(8, 8) * V
    achieved = alg_bytes / (us_launch * 1e-6) / 1e9
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
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "bri_apply FP64 1-RHS (stencil_kernel<LinkF64,nsplit,false,EPI_PLAIN>)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None,
            "us_per_launch": us_launch,
            "alg_bytes_per_launch": alg_bytes,
        },
        "bri_apply_fp64_GBps": achieved,
    }
    if not args.no_cpu:
        print("[bench] CPU oracle sample ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(L, U_np, st.shift_iters, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
