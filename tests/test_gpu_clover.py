"""GPU parity of the clover term (c_SW != 0 in eqs. (def_wils), (def_bril)) through the C ABI:
the clover field bri_build_links appends to the link array against the oracle's (built from U
with its own sigma matrices), the Brillouin and Wilson applies with the term (one and several
right-hand sides, adjoint, antiperiodic, FP32 links), and the clover-improved overlap against
the oracle's per-shift evaluation (1e-10)."""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import field, need_gpu, rel_l2

pytestmark = pytest.mark.gpu

CSW = 1.0


def _W(L, U, prec=bri.F64, tbc=0, csw=CSW):
    return bri.build_links(L, bri.links_to_device(U), prec, tbc=tbc, csw=csw)


@pytest.mark.parametrize("L,kind,tbc", [((4, 4, 4, 4), "rough", 0), ((4, 8, 4, 6), "rough", 1),
                                        ((8, 8, 8, 8), "cfg2", 0), ((2, 2, 2, 8), "rough", 1)])
def test_clover_field(L, kind, tbc):
    need_gpu()
    U, Wo = field(L, kind, tbc)
    W = _W(L, U, tbc=tbc)
    assert tuple(W.shape) == (48, 3, 3, int(np.prod(L)))
    got = bri.clover_to_host(W)
    want = oracle.clover_field(L, U, CSW)
    assert np.abs(got - want).max() <= 1e-14 * max(1.0, np.abs(want).max())
    # the link slabs themselves are those of the plain build
    W0 = bri.links_W_to_host(_W(L, U, tbc=tbc, csw=0.0))
    assert np.array_equal(bri.links_W_to_host(W)[:, :40], W0)


@pytest.mark.parametrize("kernel", ["bri", "wil"])
@pytest.mark.parametrize("L,kind,tbc", [((4, 4, 4, 4), "rough", 0), ((4, 8, 4, 6), "rough", 1),
                                        ((2, 2, 2, 8), "rough", 1)])
@pytest.mark.parametrize("dag", [False, True])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_clover_apply_f64(kernel, L, kind, tbc, dag, nrhs):
    need_gpu()
    U, Wo = field(L, kind, tbc)
    W = _W(L, U, tbc=tbc)
    C = oracle.clover_field(L, U, CSW)
    K = oracle.BrillouinKernel(Wo, C) if kernel == "bri" else oracle.WilsonKernel(U, tbc, C)
    psi = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 70, nrhs=nrhs)
    m0 = -0.9
    if kernel == "bri":
        fn = bri.apply_dag if dag else bri.apply
    else:
        fn = bri.wilson_apply_dag if dag else bri.wilson_apply
    out = bri.spinor_to_host(fn(L, W, bri.F64, m0, bri.spinor_to_device(psi)))
    ref = (oracle.dirac_adj if dag else oracle.dirac)(L, K, m0, psi)
    assert rel_l2(out, ref) < 1e-14
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


def test_clover_apply_f32():
    need_gpu()
    L = (8, 8, 8, 8)
    U, Wo = field(L, "cfg2")
    W32 = _W(L, U, bri.F32)
    psi = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 71, nrhs=2)
    K = oracle.BrillouinKernel(Wo, oracle.clover_field(L, U, CSW))
    out = bri.spinor_to_host(bri.apply(L, W32, bri.F32, -1.0, bri.spinor_to_device(psi, bri.F32)))
    assert rel_l2(out, oracle.dirac(L, K, -1.0, psi)) < 1e-6


@pytest.mark.parametrize("kernel", [bri.KERNEL_BRILLOUIN, bri.KERNEL_WILSON])
def test_clover_overlap_4_4(kernel):
    need_gpu()
    L = (4, 4, 4, 4)
    U, Wo = field(L, "cfg1")
    C = oracle.clover_field(L, U, CSW)
    K = oracle.BrillouinKernel(Wo, C) if kernel == bri.KERNEL_BRILLOUIN else oracle.WilsonKernel(U, 0, C)
    b = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 72)
    op = bri.OverlapOp(L, _W(L, U), kl_n=6, rho=1.0, tol=1e-12, max_iter=5000, kernel=kernel)
    out, st = op.apply(bri.spinor_to_device(b))
    ref, _, _ = oracle.ov_apply(L, K, 1.0, 6, b[0], tol=1e-13)
    assert rel_l2(bri.spinor_to_host(out)[0], ref) < 1e-10, st.shift_iters
    # the clover term changes the operator
    ref0, _, _ = oracle.ov_apply(L, Wo if kernel == bri.KERNEL_BRILLOUIN else oracle.WilsonKernel(U), 1.0, 6,
                                 b[0], tol=1e-13)
    assert rel_l2(ref, ref0) > 1e-3


def test_clover_every_brillouin_config():
    """With c_SW != 0 every launch configuration the tuner may pick (1-RHS splits, R = 1..4
    right-hand sides per thread, tiles and traversals) matches the oracle, FP64 and FP32."""
    import itertools

    from tests._gpu import torch

    need_gpu()
    L = (16, 8, 8, 6)
    U = synth.random_links(L, 0.6, 4243)
    Wo = oracle.links(L, U)
    K = oracle.BrillouinKernel(Wo, oracle.clover_field(L, U, CSW))
    nrhs = 5
    psi = synth.gaussian_source(L, 4244, nrhs=nrhs)
    ref = oracle.dirac(L, K, -0.9, psi)
    trav = [(0, 0, 0, 0, 0), (16, 4, 1, 1, 4), (8, 8, 1, 1, 2)]
    for prec, tol in ((bri.F64, 1e-14), (bri.F32, 1e-6)):
        W = _W(L, U, prec)
        x = bri.spinor_to_device(psi, prec)
        try:
            for t, rpt, xcd in itertools.product(trav, (1, 2, 3, 4), (0, 1)):
                cfg = bri.StencilCfg(t[0], t[1], t[2], t[3], t[4], 4, rpt, xcd)
                bri.set_stencil_cfg(L, prec, nrhs, cfg)
                got = bri.spinor_to_host(bri.apply(L, W, prec, -0.9, x))
                assert rel_l2(got, ref) < tol, (prec, cfg.as_dict())
        finally:
            bri.set_stencil_cfg(L, prec, nrhs, None)
        del W, x
        torch.cuda.empty_cache()


@pytest.mark.parametrize("kernel", ["bri", "wil"])
def test_clover_wide_batches_match_single_launches(kernel):
    """16^3x64 has 4096 tiles, where the default multi-RHS launch carries R = 4 (8 sources) or
    R = 3 (6 sources) per thread: with the clover term, for both kernels and FP64 / FP32, every
    batched column equals the single-source launch (oracle-checked above)."""
    from tests._gpu import torch

    need_gpu()
    L = (16, 16, 16, 64)
    U = synth.random_links(L, 0.4, 4245)
    Ud = bri.links_to_device(U)
    fn = bri.apply if kernel == "bri" else bri.wilson_apply
    for prec in (bri.F64, bri.F32):
        W = bri.build_links(L, Ud, prec, csw=CSW)
        for nrhs in (8, 6):
            assert bri.get_stencil_cfg(L, prec, nrhs).rpt == (4 if nrhs == 8 else 3)
            x = bri.spinor_to_device(synth.gaussian_source(L, 4246 + nrhs, nrhs=nrhs), prec)
            out = fn(L, W, prec, -0.9, x)
            for r in range(nrhs):
                one = fn(L, W, prec, -0.9, x[r:r + 1].contiguous())
                err = float(torch.linalg.vector_norm(out[r] - one[0]) / torch.linalg.vector_norm(one[0]))
                assert err < (1e-14 if prec == bri.F64 else 1e-6), (prec, nrhs, r, err)
        del W
        torch.cuda.empty_cache()
