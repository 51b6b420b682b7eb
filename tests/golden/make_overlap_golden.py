"""Write the stored FP64 oracle outputs of the overlap apply at the full workload lattices.

D_ov psi = rho (psi + X r_n(X^dag X) psi), X = D_bri(-rho), eq. (def_over) with the partial
fractions of eq. (KLnn_parfrac), computed by the oracle alone (every shift solved by its own
textbook CG to a true residual of 1e-13, links by brute-force path enumeration).  A lattice this
size takes the oracle tens of minutes per source, so the GPU tests and the benchmark compare
against what this script stores instead of recomputing it:

  * the output at a fixed set of sites: every site within two steps of the source point
    (the point-source output is concentrated there), the face / corner / middle classes of
    every axis, and seeded random sites;
  * the global norm |D_ov psi|;
  * two projections <w_k, D_ov psi> on seeded unit Gaussian spinors w_k (synth.gaussian_source),
    which see an error anywhere on the lattice: |<w, got - ref>| <= |got - ref| for |w| = 1.

Inputs are the seeded recipes of the workloads (synth, numpy): links exp(i eps A) then three
APE steps at alpha = 0.6, periodic boundaries; sources are unit point sources at the origin or
a normalised complex Gaussian.  Only `oracle` and `synth` are used.

Usage: python tests/golden/make_overlap_golden.py CASE [CASE ...]   (cases: see CASES)
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PROJ_SEEDS = (4242, 4243)
KL_N = 16
RHO = 1.0
TOL = 1e-13

L24 = (24, 24, 24, 48)
L32 = (32, 32, 32, 64)

# name: (lattice, eps, link seed, source kind, source argument)
CASES = {
    "24x24x24x48_point0": (L24, 0.7, synth.LINK_SEED_BASE + 3, "point", 0),
    "24x24x24x48_gauss": (L24, 0.7, synth.LINK_SEED_BASE + 3, "gauss", synth.SOURCE_SEED_BASE + 3),
    "32x32x32x64_point0": (L32, 0.7, synth.LINK_SEED_BASE + 4, "point", 0),
    "32x32x32x64_point7": (L32, 0.7, synth.LINK_SEED_BASE + 4, "point", 7),
    "32x32x32x64_point11": (L32, 0.7, synth.LINK_SEED_BASE + 4, "point", 11),
}


def path(name: str) -> str:
    return os.path.join(HERE, f"overlap_{name}.npz")


def sample_sites(L, seed: int, n_random: int = 256) -> np.ndarray:
    """Sites within two steps (per axis) of the origin, the classes {0, 1, L/2 - 1, L/2, L - 2, L - 1}
    on every axis, and n_random seeded random sites; sorted, unique."""
    Lx, Ly, Lz, Lt = L
    near = [-2, -1, 0, 1, 2]
    out = set()
    for t in near:
        for z in near:
            for y in near:
                for x in near:
                    c = (x % Lx, y % Ly, z % Lz, t % Lt)
                    out.add(c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3])))
    cls = [lambda n: 0, lambda n: 1, lambda n: n // 2 - 1, lambda n: n // 2, lambda n: n - 2, lambda n: n - 1]
    rng = np.random.default_rng(seed)
    for _ in range(256):
        c = [cls[rng.integers(0, len(cls))](n) for n in L]
        out.add(c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3])))
    V = Lx * Ly * Lz * Lt
    out.update(int(v) for v in rng.integers(0, V, n_random))
    return np.array(sorted(out), dtype=np.int64)


def source(L, kind: str, arg: int) -> np.ndarray:
    if kind == "point":
        return synth.point_sources_12(L)[arg]
    return synth.gaussian_source(L, arg)[0]


def make(name: str) -> None:
    L, eps, seed, kind, arg = CASES[name]
    t0 = time.time()
    print(f"[{name}] links: exp(i {eps} A) seed {seed} + 3 APE(0.6) on {L}", flush=True)
    U = synth.smeared_links(L, eps, seed, 0.6, 3)
    W = oracle.links(L, U, tbc=0)
    del U
    b = source(L, kind, arg)
    print(f"[{name}] oracle ov_apply [{KL_N}/{KL_N}], {oracle.num_threads()} threads "
          f"({time.time() - t0:.0f} s so far)", flush=True)
    t1 = time.time()
    out, iters, rel = oracle.ov_apply(L, W, RHO, KL_N, b, tol=TOL)
    t_apply = time.time() - t1
    del W
    sites = sample_sites(L, seed)
    proj = np.array([np.vdot(synth.gaussian_source(L, s)[0].ravel(), out.ravel()) for s in PROJ_SEEDS])
    np.savez_compressed(
        path(name),
        L=np.array(L, dtype=np.int64), eps=eps, link_seed=seed, ape_alpha=0.6, ape_steps=3, tbc=0,
        source_kind=kind, source_arg=arg, kl_n=KL_N, rho=RHO, tol=TOL,
        sites=sites, out_sites=out[sites], norm=float(np.linalg.norm(out.ravel())),
        proj_seeds=np.array(PROJ_SEEDS, dtype=np.int64), proj=proj,
        shift_iters=iters, shift_rel_resid=rel, oracle_seconds=t_apply, oracle_threads=oracle.num_threads(),
    )
    print(f"[{name}] done: {t_apply:.0f} s for the apply, shift iterations {list(iters)}, "
          f"max true residual {rel.max():.1e}, |out| = {np.linalg.norm(out.ravel()):.6e}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        if n not in CASES:
            raise SystemExit(f"unknown case {n}; known: {', '.join(CASES)}")
    for n in names:
        make(n)
