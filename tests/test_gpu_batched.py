"""GPU parity of the many-right-hand-side paths against the oracle:
the RHS-blocked stencil (link entries loaded once per group of right-hand
sides, App. C.3), the batched multi-shift overlap apply (12 spin-colour point
sources), and the mixed-precision apply (FP32 or bfloat16-link inner
multi-shift with FP64 defect correction of every shift).

Tolerances: FP64 stencil 1e-14 relative (L2); FP32 / BF16-link stencil 2e-6
against the oracle on the same rounded inputs; every overlap result 1e-10
relative (L2) against the FP64 oracle."""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import field, need_gpu, rel_l2, round_links, torch
from tests._lattice import disp, shift_index

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _full_links(L, W40):
    W = np.zeros((W40.shape[0], 81, 3, 3), dtype=np.complex128)
    W[:, :40] = W40
    W[:, 40] = np.eye(3)
    for j in range(40):
        W[shift_index(L, disp(j)), 80 - j] = np.conj(np.swapaxes(W40[:, j], -1, -2))
    return W


@pytest.mark.parametrize("nrhs", [4, 5, 12])
@pytest.mark.parametrize("dag", [False, True])
def test_mrhs_stencil_f64(nrhs, dag):
    need_gpu()
    L = (8, 8, 8, 8)
    U, Wo = field(L, "cfg2")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    psi = synth.gaussian_source(L, 900 + nrhs, nrhs=nrhs)
    fn = bri.apply_dag if dag else bri.apply
    out = bri.spinor_to_host(fn(L, W, bri.F64, -1.0, bri.spinor_to_device(psi)))
    ref = (oracle.dirac_adj if dag else oracle.dirac)(L, Wo, -1.0, psi)
    for r in range(nrhs):
        assert rel_l2(out[r], ref[r]) < 1e-14


@pytest.mark.parametrize("prec", [bri.F32, bri.F32_BF16W])
@pytest.mark.parametrize("nrhs", [6, 12])
def test_mrhs_stencil_low_precision(prec, nrhs):
    need_gpu()
    L = (4, 8, 4, 6)
    U, _ = field(L, "rough")
    W64 = bri.build_links(L, bri.links_to_device(U), bri.F64)
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, 950, nrhs=nrhs).astype(np.complex64).astype(np.complex128)
    out = bri.spinor_to_host(bri.apply(L, W, prec, -1.0, bri.spinor_to_device(psi, prec)))
    Wr = _full_links(L, round_links(bri.links_W_to_host(W64), prec))
    ref = oracle.dirac(L, Wr, -1.0, psi)
    for r in range(nrhs):
        assert rel_l2(out[r], ref[r]) < 2e-6


def test_batched_overlap_12_point_sources():
    """All 12 spin-colour point sources at the origin in one batched call."""
    need_gpu()
    L = (4, 4, 4, 4)
    U, Wo = field(L, "cfg1")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    op = bri.OverlapOp(L, W, kl_n=8, rho=1.0, tol=1e-12, nrhs=12)
    b = synth.point_sources_12(L)
    out, st = op.apply(bri.spinor_to_device(b))
    got = bri.spinor_to_host(out)
    for r in (0, 5, 11):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < TOL, r
    # every column equals its own single-column apply bit for bit? no: but to 1e-13
    op1 = bri.OverlapOp(L, W, kl_n=8, rho=1.0, tol=1e-12)
    one, _ = op1.apply(bri.spinor_to_device(b[7:8]))
    assert rel_l2(got[7], bri.spinor_to_host(one)[0]) < 1e-12


@pytest.mark.parametrize("inner", [bri.F32, bri.F32_BF16W])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_mixed_precision_overlap(inner, nrhs):
    need_gpu()
    L = (4, 8, 4, 6)
    U = synth.smeared_links(L, 0.7, 1703, 0.6, 3)
    Wo = oracle.links(L, U)
    Ud = bri.links_to_device(U)
    W64 = bri.build_links(L, Ud, bri.F64)
    Wlo = bri.build_links(L, Ud, inner)
    n = 8
    op = bri.OverlapOp(L, W64, kl_n=n, rho=1.0, tol=1e-12, Wlo=Wlo, inner=inner, nrhs=nrhs)
    b = synth.gaussian_source(L, 960, nrhs=nrhs)
    out, st = op.apply(bri.spinor_to_device(b))
    got = bri.spinor_to_host(out)
    # FP32 takes over at |r| <= 1e-12 / 2^-24 |b|, bfloat16 links only at 2.6e-10 |b|
    assert st.refine >= (1 if inner == bri.F32 else 0) and max(st.rel_resid) <= 1e-12
    for r in range(nrhs):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, n, b[r], tol=1e-13)
        assert rel_l2(got[r], ref) < TOL, (r, st.refine)
    s_out, _ = op.sign(bri.spinor_to_device(b[:1]))
    sref, _, _ = oracle.sign_apply(L, Wo, 1.0, n, b[0], tol=1e-13)
    assert rel_l2(bri.spinor_to_host(s_out)[0], sref) < TOL


@pytest.mark.parametrize("inner", [bri.F32, bri.F32_BF16W])
def test_mixed_iteration_cap_reports_noconv(inner):
    need_gpu()
    L = (4, 4, 4, 4)
    U, _ = field(L, "cfg1")
    Ud = bri.links_to_device(U)
    W64 = bri.build_links(L, Ud, bri.F64)
    Wlo = bri.build_links(L, Ud, inner)
    op = bri.OverlapOp(L, W64, kl_n=8, tol=1e-13, max_iter=6, Wlo=Wlo, inner=inner)
    out, st = op.apply(bri.spinor_to_device(synth.point_source(L)), allow_noconv=True)
    assert st.status == bri.ENOCONV and st.iters <= 6 and max(st.rel_resid) > 1e-13


def test_mixed_precision_33_columns():
    """33 sources: the FP64 batch against the oracle, and the mixed-precision batch against FP64."""
    need_gpu()
    L = (4, 4, 4, 4)
    U, Wo = field(L, "cfg1")
    Ud = bri.links_to_device(U)
    W64 = bri.build_links(L, Ud, bri.F64)
    Wlo = bri.build_links(L, Ud, bri.F32)
    n, nrhs = 8, 33
    b = synth.gaussian_source(L, 961, nrhs=nrhs)
    bd = bri.spinor_to_device(b)
    out64, st64 = bri.OverlapOp(L, W64, kl_n=n, tol=1e-12, nrhs=nrhs).apply(bd)
    outm, stm = bri.OverlapOp(L, W64, kl_n=n, tol=1e-12, Wlo=Wlo, inner=bri.F32, nrhs=nrhs).apply(bd)
    g64, gm = bri.spinor_to_host(out64), bri.spinor_to_host(outm)
    for r in (0, 16, 32):
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, n, b[r], tol=1e-13)
        assert rel_l2(g64[r], ref) < TOL, r
    for r in range(nrhs):
        assert rel_l2(gm[r], g64[r]) < TOL, (r, stm.refine)
    assert stm.refine >= 1 and max(stm.rel_resid) <= 1e-12 and max(st64.rel_resid) <= 1e-12
