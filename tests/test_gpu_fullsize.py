"""Parity at the full lattice sizes of the workloads: 24^3x48 (mixed-precision overlap,
links exp(0.7 i A) + 3 APE steps) and 32^3x64 (12 spin-colour point sources x 16 shifts), and
at 48^3x96, whose link array is past 32-bit element offsets.

The oracle cannot hold the link array of these lattices, so the stencil is checked at
sampled sites (every face and corner class plus random sites) against the oracle's
per-site sums with links built on the fly (App. C.1, eq. (def_bril)); the overlap apply,
whose value at one site depends on the whole lattice, is checked through properties that
hold at any size: sign(H)^2 = 1 and the Ginsparg-Wilson identity to the rational's
accuracy, batched columns against single-source applies, and the mixed-precision solves
against FP64 to 1e-10 per source.

Tolerances: FP64 stencil 1e-13 of the largest entry; FP32 / bfloat16-link stencils 1e-5 /
2e-2 of it (rounded links and spinors, 81-term FP32 sums).
"""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, torch

pytestmark = pytest.mark.gpu

L24 = (24, 24, 24, 48)
L32 = (32, 32, 32, 64)


def _links(L, eps, seed):
    U = synth.smeared_links_torch(L, eps, seed, 0.6, 3, device="cuda", chunk=1 << 18)  # (4, V, 3, 3)
    return U, U.permute(0, 2, 3, 1).contiguous()


def _sites(L, rng, n_random=24):
    out = []
    for cx in (0, L[0] - 1):
        for cy in (0, L[1] // 2):
            for cz in (0, L[2] - 1):
                for ct in (0, L[3] - 1, L[3] // 2):
                    out.append(cx + L[0] * (cy + L[1] * (cz + L[2] * ct)))
    V = int(np.prod(L))
    out += [int(v) for v in rng.integers(0, V, n_random)]
    return out


def _rel(r):
    return 1 / float(np.abs(r).max())


@pytest.mark.parametrize("L,eps,seed", [(L24, 0.7, synth.LINK_SEED_BASE + 3), (L32, 0.7, synth.LINK_SEED_BASE + 4)])
def test_stencil_sampled_sites(L, eps, seed):
    need_gpu()
    U, Ud = _links(L, eps, seed)
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    psi = synth.gaussian_source(L, seed + 1)  # (1, V, 4, 3)
    sites = _sites(L, rng)
    Uh = U.cpu().numpy()
    del U
    m0 = -1.0
    ref = oracle.dirac_at(L, Uh, 1, m0, psi[0], sites)
    refd = oracle.dirac_adj_at(L, Uh, 1, m0, psi[0], sites)
    scale, scaled = np.abs(ref).max(), np.abs(refd).max()
    for prec, tol in ((bri.F64, 1e-13), (bri.F32, 1e-5), (bri.F32_BF16W, 2e-2)):
        W = bri.build_links(L, Ud, prec, tbc=1)
        p = bri.spinor_to_device(psi, prec)
        out = bri.apply(L, W, prec, m0, p)[0]
        outd = bri.apply_dag(L, W, prec, m0, p)[0]
        idx = torch.tensor(sites, device="cuda")
        got = out[:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
        gotd = outd[:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
        assert np.abs(got - ref).max() <= tol * scale, prec
        assert np.abs(gotd - refd).max() <= tol * scaled, prec
        del W, p, out, outd
    torch.cuda.empty_cache()


def test_batched_defaults_sampled_sites_32_64():
    """The batch defaults on the benchmark lattice (whole-line tiles in columns of 4 z-slices, the
    column groups of a tile in consecutive blocks: FP64 R = 2, FP32 R = 3 two rows wide, bfloat16
    links the x-line kernel one RHS per thread) on 5 columns (ragged groups), every column against
    the oracle at sampled sites (App. C.1 stencil), D and D^dag."""
    need_gpu()
    L = L32
    seed = synth.LINK_SEED_BASE + 6
    U, Ud = _links(L, 0.7, seed)
    rng = np.random.default_rng(seed)
    nrhs = 5
    psi = synth.gaussian_source(L, seed + 1, nrhs=nrhs)
    sites = _sites(L, rng, n_random=8)
    Uh = U.cpu().numpy()
    del U
    m0 = -1.0
    ref = [oracle.dirac_at(L, Uh, 0, m0, psi[c], sites) for c in range(nrhs)]
    refd = [oracle.dirac_adj_at(L, Uh, 0, m0, psi[c], sites) for c in range(nrhs)]
    idx = torch.tensor(sites, device="cuda")
    for prec, tol in ((bri.F64, 1e-13), (bri.F32, 1e-5), (bri.F32_BF16W, 2e-2)):
        cfg = bri.get_stencil_cfg(L, prec, nrhs)
        assert (cfg.tile_x, cfg.col_z) == (32, 4), cfg.as_dict()
        print(f"[fullsize] batch defaults prec {prec}: {cfg.as_dict()}", flush=True)
        W = bri.build_links(L, Ud, prec)
        p = bri.spinor_to_device(psi, prec)
        out = bri.apply(L, W, prec, m0, p)
        outd = bri.apply_dag(L, W, prec, m0, p)
        for c in range(nrhs):
            got = out[c][:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
            gotd = outd[c][:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
            assert np.abs(got - ref[c]).max() <= tol * np.abs(ref[c]).max(), (prec, c)
            assert np.abs(gotd - refd[c]).max() <= tol * np.abs(refd[c]).max(), (prec, c)
        del W, p, out, outd
        torch.cuda.empty_cache()


def _identities(op, b, tol):
    s1, st1 = op.sign(b)
    s2, _ = op.sign(s1)
    assert float(torch.linalg.vector_norm(s2 - b) / torch.linalg.vector_norm(b)) < tol
    g5 = torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=torch.float64, device=b.device).view(1, 4, 1, 1)
    Db, _ = op.apply(b)
    Dg5b, _ = op.apply(b * g5)
    Dg5Db, _ = op.apply(Db * g5)
    gw = Dg5b + g5 * Db - Dg5Db  # Ginsparg-Wilson with rho = 1
    assert float(torch.linalg.vector_norm(gw) / torch.linalg.vector_norm(b)) < tol
    return Db, st1


def test_mixed_precision_overlap_24_48():
    need_gpu()
    L = L24
    _, Ud = _links(L, 0.7, synth.LINK_SEED_BASE + 3)
    W = bri.build_links(L, Ud, bri.F64)
    b = bri.spinor_to_device(synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 3))
    op = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000)
    ref, st = _identities(op, b, 1e-9)
    assert 10 < st.iters < 2000
    del op
    for inner in (bri.F32, bri.F32_BF16W):
        Wlo = bri.build_links(L, Ud, inner)
        opm = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000, Wlo=Wlo, inner=inner)
        out, stm = opm.apply(b)
        err = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
        assert err < 1e-10, (inner, err, stm.refine)
        assert max(stm.rel_resid) <= 1e-12
        del opm, Wlo
        torch.cuda.empty_cache()


def test_batched_point_sources_32_64():
    need_gpu()
    L = L32
    _, Ud = _links(L, 0.7, synth.LINK_SEED_BASE + 4)
    W = bri.build_links(L, Ud, bri.F64)
    b12 = bri.spinor_to_device(synth.point_sources_12(L))
    op12 = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000, nrhs=12)
    out12, st12 = op12.apply(b12)
    assert max(st12.rel_resid) <= 1e-12
    del op12
    torch.cuda.empty_cache()
    op1 = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000)
    for r in (0, 7):
        o1, _ = op1.apply(b12[r:r + 1].contiguous())
        err = float(torch.linalg.vector_norm(o1[0] - out12[r]) / torch.linalg.vector_norm(o1[0]))
        assert err < 1e-11, (r, err)
    _identities(op1, b12[5:6].contiguous(), 1e-9)
    del op1
    torch.cuda.empty_cache()
    # mixed precision on four of the sources, batched, against the FP64 batched result
    Wlo = bri.build_links(L, Ud, bri.F32)
    opm = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000, Wlo=Wlo, inner=bri.F32, nrhs=4)
    sel = [0, 4, 8, 11]
    om, stm = opm.apply(b12[sel].contiguous())
    for k, r in enumerate(sel):
        err = float(torch.linalg.vector_norm(om[k] - out12[r]) / torch.linalg.vector_norm(out12[r]))
        assert err < 1e-10, (r, err)
    del opm, Wlo
    torch.cuda.empty_cache()


def test_lattice_past_32_bit_link_offsets_48_96():
    """48^3x96, 10.6 M sites: the FP64 link array holds 360 V = 3.8e9 complex entries (61 GB),
    past 32-bit element offsets.  The FP64 and FP32 stencils and their adjoints at sampled sites
    against the oracle, then sign(H)^2 = 1 and Ginsparg-Wilson through the overlap apply."""
    need_gpu()
    L = (48, 48, 48, 96)
    seed = synth.LINK_SEED_BASE + 5
    U, Ud = _links(L, 0.7, seed)
    rng = np.random.default_rng(seed)
    psi = synth.gaussian_source(L, seed + 1)
    sites = _sites(L, rng, n_random=16)
    Uh = U.cpu().numpy()
    del U
    m0 = -1.0
    ref = oracle.dirac_at(L, Uh, 0, m0, psi[0], sites)
    refd = oracle.dirac_adj_at(L, Uh, 0, m0, psi[0], sites)
    del Uh
    scale, scaled = np.abs(ref).max(), np.abs(refd).max()
    idx = torch.tensor(sites, device="cuda")
    for prec, tol in ((bri.F32, 1e-5), (bri.F64, 1e-13)):
        W = bri.build_links(L, Ud, prec)
        p = bri.spinor_to_device(psi, prec)
        got = bri.apply(L, W, prec, m0, p)[0][:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
        gotd = bri.apply_dag(L, W, prec, m0, p)[0][:, :, idx].permute(2, 0, 1).cpu().numpy().astype(np.complex128)
        assert np.abs(got - ref).max() <= tol * scale, prec
        assert np.abs(gotd - refd).max() <= tol * scaled, prec
        del p
        if prec == bri.F32:
            del W
            torch.cuda.empty_cache()
    del Ud
    b = bri.spinor_to_device(psi)
    op = bri.OverlapOp(L, W, kl_n=16, tol=1e-12, max_iter=5000)
    _, st = _identities(op, b, 1e-9)
    assert 10 < st.iters < 2000
    del op, W, b
    torch.cuda.empty_cache()
