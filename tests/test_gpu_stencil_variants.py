"""The stencil kernel variants compute the Brillouin operator of App. C.1 exactly as the
standard launch does:
  * t-streaming (a block walks the t-slices of its xyz tile and reads both uses of every stored
    link inside one slice): every streaming tiling, chunk lengths from one slice to the whole t
    extent (the last chunk wraps to slice 0);
  * x-line (tiles spanning whole x-lines; the three x-displacements of each (dy, dz, dt) share one
    spinor load and reach the neighbours by cross-lane moves): x extents 1, 2, 8, 16, 32, 64, both
    traversals, 1, 2 and 4 waves per tile;
checked through bri_apply / bri_apply_dag against the oracle's direct 81-term sum, for several
columns, degenerate extents, low precision, the clover term, antiperiodic links, and the fused
solver epilogues (norms, CG residual update, overlap and sign outputs) through the overlap apply
against the oracle's eq. (def_over) with every shift solved on its own."""

import itertools

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, rel_l2

pytestmark = pytest.mark.gpu

L = (16, 8, 8, 6)


def _stream_cfgs(L):
    tiles = [(16, 8, 2), (8, 8, 4), (16, 4, 4), (4, 8, 8), (16, 16, 1), (32, 8, 1)]
    for (tx, ty, tz), ct, xcd in itertools.product(tiles, (1, 2, 3, 6, 4), (0, 1)):
        if L[0] % tx or L[1] % ty or L[2] % tz or L[3] % ct:
            continue
        yield bri.StencilCfg(tx, ty, tz, ct, 0, 1, 0, xcd, 1)  # variant 1: t-streaming


@pytest.fixture(scope="module")
def field():
    U = synth.random_links(L, 0.6, 4243)
    return U, oracle.links(L, U), bri.build_links(L, bri.links_to_device(U), bri.F64)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_stream_configs_match_oracle(field, nrhs):
    need_gpu()
    _, Wo, W = field
    psi = synth.gaussian_source(L, 61 + nrhs, nrhs=nrhs)
    ref = oracle.dirac(L, Wo, -0.9, psi)
    refd = oracle.dirac_adj(L, Wo, -0.9, psi)
    x = bri.spinor_to_device(psi)
    n = 0
    try:
        for cfg in _stream_cfgs(L):
            bri.set_stencil_cfg(L, bri.F64, nrhs, cfg)
            got = bri.spinor_to_host(bri.apply(L, W, bri.F64, -0.9, x))
            gotd = bri.spinor_to_host(bri.apply_dag(L, W, bri.F64, -0.9, x))
            for r in range(nrhs):
                assert rel_l2(got[r], ref[r]) < 1e-14, cfg.as_dict()
                assert rel_l2(gotd[r], refd[r]) < 1e-14, cfg.as_dict()
            n += 1
    finally:
        bri.set_stencil_cfg(L, bri.F64, nrhs, None)
    assert n >= 12


@pytest.mark.parametrize("Ld,cfg", [
    ((16, 16, 1, 4), (16, 16, 1, 2)),   # z extent 1: the z neighbours are the site itself
    ((8, 16, 2, 2), (8, 16, 2, 1)),     # z extent 2 and one-slice chunks
    ((16, 8, 4, 1), (16, 4, 4, 1)),     # t extent 1: slices s - 1 and s + 1 are s
])
def test_stream_degenerate_extents(Ld, cfg):
    need_gpu()
    U = synth.random_links(Ld, 0.5, 4244)
    Wo = oracle.links(Ld, U)
    W = bri.build_links(Ld, bri.links_to_device(U), bri.F64)
    psi = synth.gaussian_source(Ld, 65)
    x = bri.spinor_to_device(psi)
    c = bri.StencilCfg(cfg[0], cfg[1], cfg[2], cfg[3], 0, 1, 0, 1, 1)
    try:
        bri.set_stencil_cfg(Ld, bri.F64, 1, c)
        got = bri.spinor_to_host(bri.apply(Ld, W, bri.F64, -0.7, x))[0]
        gotd = bri.spinor_to_host(bri.apply_dag(Ld, W, bri.F64, -0.7, x))[0]
    finally:
        bri.set_stencil_cfg(Ld, bri.F64, 1, None)
    assert rel_l2(got, oracle.dirac(Ld, Wo, -0.7, psi[0])) < 1e-14
    assert rel_l2(gotd, oracle.dirac_adj(Ld, Wo, -0.7, psi[0])) < 1e-14


@pytest.mark.parametrize("prec,tol", [(bri.F32, 2e-6), (bri.F32_BF16W, 2e-2)])
def test_stream_low_precision(field, prec, tol):
    need_gpu()
    U, Wo, _ = field
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, 66)
    x = bri.spinor_to_device(psi, prec)
    try:
        bri.set_stencil_cfg(L, prec, 1, bri.StencilCfg(8, 8, 4, 3, 0, 1, 0, 1, 1))
        got = bri.spinor_to_host(bri.apply(L, W, prec, -0.9, x))[0]
    finally:
        bri.set_stencil_cfg(L, prec, 1, None)
    assert rel_l2(got, oracle.dirac(L, Wo, -0.9, psi[0])) < tol


def test_stream_clover_antiperiodic():
    need_gpu()
    U = synth.random_links(L, 0.5, 4245)
    csw = 1.0
    Wo = oracle.BrillouinKernel(oracle.links(L, U, tbc=1), oracle.clover_field(L, U, csw))
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=1, csw=csw)
    psi = synth.gaussian_source(L, 67)
    x = bri.spinor_to_device(psi)
    try:
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(16, 8, 2, 2, 0, 1, 0, 1, 1))
        got = bri.spinor_to_host(bri.apply(L, W, bri.F64, -0.8, x))[0]
        gotd = bri.spinor_to_host(bri.apply_dag(L, W, bri.F64, -0.8, x))[0]
    finally:
        bri.set_stencil_cfg(L, bri.F64, 1, None)
    assert rel_l2(got, oracle.dirac(L, Wo, -0.8, psi[0])) < 1e-14
    assert rel_l2(gotd, oracle.dirac_adj(L, Wo, -0.8, psi[0])) < 1e-14


@pytest.mark.parametrize("nrhs", [1, 2])
def test_stream_solver_epilogues(field, nrhs):
    """The overlap apply and sign function with the streaming kernel installed for the
    solve's column count: norms, CG residual update, overlap and sign epilogues."""
    need_gpu()
    _, Wo, W = field
    b = synth.gaussian_source(L, 68, nrhs=nrhs)
    try:
        bri.set_stencil_cfg(L, bri.F64, nrhs, bri.StencilCfg(8, 8, 4, 2, 0, 1, 0, 1, 1))
        op = bri.OverlapOp(L, W, kl_n=8, tol=1e-12, nrhs=nrhs)
        out, st = op.apply(bri.spinor_to_device(b))
        sgn, _ = op.sign(bri.spinor_to_device(b))
    finally:
        bri.set_stencil_cfg(L, bri.F64, nrhs, None)
    got, gots = bri.spinor_to_host(out), bri.spinor_to_host(sgn)
    for r in range(nrhs):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        refs, _, _ = oracle.sign_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < 1e-10
        assert rel_l2(gots[r], refs) < 1e-10
    assert max(st.rel_resid) <= 1e-12


# ---------------------------------------------------------------- x-line variant

def _xline_cfgs(L):
    """(tile, colz) choices whose tile spans the x extent, nsplit 1/2/4, xcd 0/1."""
    out = []
    tx = L[0]
    for ty in (1, 2, 4, 8, 16, 32, 64):
        for tz in (1, 2, 4, 8):
            for tt in (1, 2, 4):
                if tx * ty * tz * tt != 64 or L[1] % ty or L[2] % tz or L[3] % tt:
                    continue
                out.append(((tx, ty, tz, tt), 0))
                if tz == 1 and tt == 1:
                    out += [((tx, ty, 1, 1), cz) for cz in (2, 4) if L[2] % cz == 0]
    for (t, cz), ns, xcd in itertools.product(out, (1, 2, 4), (0, 1)):
        yield bri.StencilCfg(t[0], t[1], t[2], t[3], cz, ns, 0, xcd, 2)
    for (t, cz), rpt in itertools.product(out[:3], (2, 3, 4)):  # R right-hand sides per thread
        yield bri.StencilCfg(t[0], t[1], t[2], t[3], cz, 4, rpt, 1, 2)


@pytest.mark.parametrize("Lx", [(16, 8, 8, 6), (32, 4, 4, 4), (64, 2, 2, 4), (8, 8, 4, 4), (2, 8, 4, 4),
                                (1, 8, 8, 8)])
def test_xline_configs_match_oracle(Lx):
    need_gpu()
    U = synth.random_links(Lx, 0.6, 4246)
    Wo = oracle.links(Lx, U)
    W = bri.build_links(Lx, bri.links_to_device(U), bri.F64)
    nrhs = 5  # a partial last group of columns for 2, 3 and 4 per thread
    psi = synth.gaussian_source(Lx, 69, nrhs=nrhs)
    ref = oracle.dirac(Lx, Wo, -0.9, psi)
    refd = oracle.dirac_adj(Lx, Wo, -0.9, psi)
    x = bri.spinor_to_device(psi)
    n = 0
    try:
        for cfg in _xline_cfgs(Lx):
            bri.set_stencil_cfg(Lx, bri.F64, nrhs, cfg)
            got = bri.spinor_to_host(bri.apply(Lx, W, bri.F64, -0.9, x))
            gotd = bri.spinor_to_host(bri.apply_dag(Lx, W, bri.F64, -0.9, x))
            for r in range(nrhs):
                assert rel_l2(got[r], ref[r]) < 1e-14, cfg.as_dict()
                assert rel_l2(gotd[r], refd[r]) < 1e-14, cfg.as_dict()
            n += 1
    finally:
        bri.set_stencil_cfg(Lx, bri.F64, nrhs, None)
    assert n >= 6


def test_xline_rejects_partial_lines(field):
    need_gpu()
    with pytest.raises(bri.BriError):
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(8, 8, 1, 1, 2, 4, 0, 1, 2))


@pytest.mark.parametrize("prec,tol", [(bri.F32, 2e-6), (bri.F32_BF16W, 2e-2)])
def test_xline_low_precision(field, prec, tol):
    need_gpu()
    U, Wo, _ = field
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, 70)
    x = bri.spinor_to_device(psi, prec)
    try:
        bri.set_stencil_cfg(L, prec, 1, bri.StencilCfg(16, 4, 1, 1, 4, 4, 0, 1, 2))
        got = bri.spinor_to_host(bri.apply(L, W, prec, -0.9, x))[0]
    finally:
        bri.set_stencil_cfg(L, prec, 1, None)
    assert rel_l2(got, oracle.dirac(L, Wo, -0.9, psi[0])) < tol


def test_xline_clover_antiperiodic():
    need_gpu()
    U = synth.random_links(L, 0.5, 4247)
    csw = 1.0
    Wo = oracle.BrillouinKernel(oracle.links(L, U, tbc=1), oracle.clover_field(L, U, csw))
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=1, csw=csw)
    psi = synth.gaussian_source(L, 71)
    x = bri.spinor_to_device(psi)
    try:
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(16, 4, 1, 1, 2, 2, 0, 1, 2))
        got = bri.spinor_to_host(bri.apply(L, W, bri.F64, -0.8, x))[0]
        gotd = bri.spinor_to_host(bri.apply_dag(L, W, bri.F64, -0.8, x))[0]
    finally:
        bri.set_stencil_cfg(L, bri.F64, 1, None)
    assert rel_l2(got, oracle.dirac(L, Wo, -0.8, psi[0])) < 1e-14
    assert rel_l2(gotd, oracle.dirac_adj(L, Wo, -0.8, psi[0])) < 1e-14


@pytest.mark.parametrize("nrhs", [1, 3])
def test_xline_solver_epilogues(field, nrhs):
    need_gpu()
    _, Wo, W = field
    b = synth.gaussian_source(L, 72, nrhs=nrhs)
    try:
        bri.set_stencil_cfg(L, bri.F64, nrhs, bri.StencilCfg(16, 4, 1, 1, 4, 4, 0, 1, 2))
        op = bri.OverlapOp(L, W, kl_n=8, tol=1e-12, nrhs=nrhs)
        out, st = op.apply(bri.spinor_to_device(b))
        sgn, _ = op.sign(bri.spinor_to_device(b))
    finally:
        bri.set_stencil_cfg(L, bri.F64, nrhs, None)
    got, gots = bri.spinor_to_host(out), bri.spinor_to_host(sgn)
    for r in range(nrhs):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        refs, _, _ = oracle.sign_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < 1e-10
        assert rel_l2(gots[r], refs) < 1e-10
    assert max(st.rel_resid) <= 1e-12


@pytest.mark.parametrize("prec,tol", [(bri.F32, 2e-6), (bri.F32_BF16W, 2e-2)])
@pytest.mark.parametrize("rpt", [2, 3, 4])
def test_xline_mrhs_low_precision(field, prec, tol, rpt):
    need_gpu()
    U, Wo, _ = field
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, 73, nrhs=7)
    x = bri.spinor_to_device(psi, prec)
    ref = oracle.dirac(L, Wo, -0.9, psi)
    refd = oracle.dirac_adj(L, Wo, -0.9, psi)
    try:
        bri.set_stencil_cfg(L, prec, 7, bri.StencilCfg(16, 4, 1, 1, 4, 4, rpt, 1, 2))
        got = bri.spinor_to_host(bri.apply(L, W, prec, -0.9, x))
        gotd = bri.spinor_to_host(bri.apply_dag(L, W, prec, -0.9, x))
    finally:
        bri.set_stencil_cfg(L, prec, 7, None)
    for r in range(7):
        assert rel_l2(got[r], ref[r]) < tol
        assert rel_l2(gotd[r], refd[r]) < tol


def test_xline_mrhs_solver_epilogues(field):
    """Batched overlap apply and sign function with the x-line multi-RHS kernel (3 per thread,
    a partial group) installed for the solve's 5 columns."""
    need_gpu()
    _, Wo, W = field
    b = synth.gaussian_source(L, 74, nrhs=5)
    try:
        bri.set_stencil_cfg(L, bri.F64, 5, bri.StencilCfg(16, 4, 1, 1, 2, 4, 3, 1, 2))
        op = bri.OverlapOp(L, W, kl_n=8, tol=1e-12, nrhs=5)
        out, st = op.apply(bri.spinor_to_device(b))
    finally:
        bri.set_stencil_cfg(L, bri.F64, 5, None)
    got = bri.spinor_to_host(out)
    for r in (0, 4):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < 1e-10
    assert max(st.rel_resid) <= 1e-12


# ------------------------------------------------------------ matrix-core variant

@pytest.mark.parametrize("prec,tol", [(bri.F32, 2e-6), (bri.F32_BF16W, 2e-2)])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_mfma_configs_match_oracle(field, prec, tol, nrhs):
    """The FP32-MFMA transport: every right-hand-side count per thread (a partial last group
    with 5 columns), both traversals, against the oracle's 81-term sum."""
    need_gpu()
    U, Wo, _ = field
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, 75 + nrhs, nrhs=nrhs)
    x = bri.spinor_to_device(psi, prec)
    ref = oracle.dirac(L, Wo, -0.9, psi)
    refd = oracle.dirac_adj(L, Wo, -0.9, psi)
    n = 0
    try:
        for (t, cz), rpt in itertools.product([((16, 4, 1, 1), 2), ((0, 0, 0, 0), 0), ((4, 4, 4, 1), 0)],
                                              (1, 2, 3, 4)):
            if rpt > 1 and nrhs == 1:
                continue
            bri.set_stencil_cfg(L, prec, nrhs, bri.StencilCfg(t[0], t[1], t[2], t[3], cz, 4, rpt, 1, 3))
            got = bri.spinor_to_host(bri.apply(L, W, prec, -0.9, x))
            gotd = bri.spinor_to_host(bri.apply_dag(L, W, prec, -0.9, x))
            for r in range(nrhs):
                assert rel_l2(got[r], ref[r]) < tol, (rpt, t)
                assert rel_l2(gotd[r], refd[r]) < tol, (rpt, t)
            n += 1
    finally:
        bri.set_stencil_cfg(L, prec, nrhs, None)
    assert n >= 3


def test_mfma_rejected_for_fp64(field):
    need_gpu()
    _, _, W = field
    x = bri.spinor_to_device(synth.gaussian_source(L, 80))
    with pytest.raises(bri.BriError):
        bri.stencil_time(L, W, bri.F64, x, cfg=bri.StencilCfg(16, 4, 1, 1, 2, 4, 1, 1, 3), reps=1)


def test_mfma_clover():
    need_gpu()
    U = synth.random_links(L, 0.5, 4248)
    csw = 1.0
    Wo = oracle.BrillouinKernel(oracle.links(L, U), oracle.clover_field(L, U, csw))
    W = bri.build_links(L, bri.links_to_device(U), bri.F32, csw=csw)
    psi = synth.gaussian_source(L, 81, nrhs=3)
    x = bri.spinor_to_device(psi, bri.F32)
    try:
        bri.set_stencil_cfg(L, bri.F32, 3, bri.StencilCfg(16, 4, 1, 1, 2, 4, 2, 1, 3))
        got = bri.spinor_to_host(bri.apply(L, W, bri.F32, -0.8, x))
        gotd = bri.spinor_to_host(bri.apply_dag(L, W, bri.F32, -0.8, x))
    finally:
        bri.set_stencil_cfg(L, bri.F32, 3, None)
    for r in range(3):
        assert rel_l2(got[r], oracle.dirac(L, Wo, -0.8, psi[r])) < 2e-6
        assert rel_l2(gotd[r], oracle.dirac_adj(L, Wo, -0.8, psi[r])) < 2e-6


def test_mfma_in_the_mixed_solver(field):
    """The mixed-precision batch with the MFMA stencil installed for its FP32 phase (norms and CG
    residual epilogues on FP32 vectors) against the oracle's eq. (def_over)."""
    need_gpu()
    U, Wo, W64 = field
    W32 = bri.build_links(L, bri.links_to_device(U), bri.F32)
    b = synth.gaussian_source(L, 82, nrhs=4)
    try:
        bri.set_stencil_cfg(L, bri.F32, 4, bri.StencilCfg(16, 4, 1, 1, 2, 4, 4, 1, 3))
        op = bri.OverlapOp(L, W64, kl_n=8, tol=1e-12, Wlo=W32, inner=bri.F32, nrhs=4)
        out, st = op.apply(bri.spinor_to_device(b))
    finally:
        bri.set_stencil_cfg(L, bri.F32, 4, None)
    assert st.refine >= 1
    got = bri.spinor_to_host(out)
    for r in (0, 3):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < 1e-10
