"""Launch grids whose column groups do not all fit along x: the groups of a tile run in consecutive
blocks along x (as many as grid.x allows) and the rest continue along blockIdx.y.  The environment
variable BRI_GROUPS_ALONG_X lowers that count, so that small lattices reach the split: every kernel
family and epilogue must then give the same result as the uncapped launch, bit for bit (each tile
and column does the same arithmetic and fills the same partial-sum slot), and the apply must match
the oracle (App. C.1 stencil; Sec. 3.3 multi-shift for the solver epilogues)."""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu

L = (16, 8, 8, 8)  # 128 tiles of 16 x 4 sites

# (name, precision, config): every kernel family that numbers its blocks by (tile, column group)
CONFIGS = [
    ("standard 1 RHS", bri.F64, bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 0, 2)),
    ("standard 1 RHS, 2 waves", bri.F64, bri.StencilCfg(16, 4, 1, 1, 4, 2, 0, 0, 0, 1)),
    ("x-line 1 RHS", bri.F64, bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 2, 2)),
    ("multi-RHS R = 2", bri.F64, bri.StencilCfg(16, 4, 1, 1, 2, 4, 2, 1, 0, 2)),
    ("x-line multi-RHS R = 2", bri.F64, bri.StencilCfg(16, 4, 1, 1, 2, 4, 2, 1, 2, 1)),
    ("multi-RHS R = 3 FP32", bri.F32, bri.StencilCfg(16, 4, 1, 1, 2, 4, 3, 1, 0, 2)),
    ("matrix cores R = 2 FP32", bri.F32, bri.StencilCfg(16, 4, 1, 1, 2, 4, 2, 1, 3, 0)),
]


@pytest.fixture(scope="module")
def field():
    U = synth.random_links(L, 0.5, 4471)
    Ud = bri.links_to_device(U)
    return U, {p: bri.build_links(L, Ud, p) for p in (bri.F64, bri.F32)}


@pytest.mark.parametrize("name,prec,cfg", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_split_grid_matches_unsplit(field, monkeypatch, name, prec, cfg):
    need_gpu()
    U, W = field
    nrhs = 5  # ragged: 5 columns in groups of 1, 2 or 3, split 1 or 2 groups along x
    psi = synth.gaussian_source(L, 4472, nrhs=nrhs)
    x = bri.spinor_to_device(psi, prec)
    print(f"[split] {name}", flush=True)
    try:
        bri.set_stencil_cfg(L, prec, nrhs, cfg)
        monkeypatch.delenv("BRI_GROUPS_ALONG_X", raising=False)
        ref = bri.apply(L, W[prec], prec, -0.9, x)
        refd = bri.apply_dag(L, W[prec], prec, -0.9, x)
        for cap in ("1", "2"):
            monkeypatch.setenv("BRI_GROUPS_ALONG_X", cap)
            got = bri.apply(L, W[prec], prec, -0.9, x)
            gotd = bri.apply_dag(L, W[prec], prec, -0.9, x)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (name, cap)
            assert torch.equal(gotd, refd), (name, cap)
    finally:
        bri.set_stencil_cfg(L, prec, nrhs, None)
    if prec == bri.F64:
        Wo = oracle.links(L, U)
        want = oracle.dirac(L, Wo, -0.9, psi)
        g = bri.spinor_to_host(got)
        for r in range(nrhs):
            assert rel_l2(g[r], want[r]) < 1e-14, (name, r)


def test_split_grid_in_the_multishift_solver(field, monkeypatch):
    """The fused epilogues (|t|^2, |p|^2, the r update and |r|^2, the overlap output) through a split
    grid: the batched overlap apply is identical to the unsplit one, iteration for iteration."""
    need_gpu()
    U, W = field
    b = np.concatenate([synth.gaussian_source(L, 4473), synth.point_sources_12(L)[[2, 9]]])
    bd = bri.spinor_to_device(b)
    cfg = bri.StencilCfg(16, 4, 1, 1, 2, 4, 2, 1, 0, 2)
    try:
        bri.set_stencil_cfg(L, bri.F64, 3, cfg)
        monkeypatch.delenv("BRI_GROUPS_ALONG_X", raising=False)
        op = bri.OverlapOp(L, W[bri.F64], kl_n=8, rho=1.0, tol=1e-12, nrhs=3)
        ref, st_ref = op.apply(bd)
        monkeypatch.setenv("BRI_GROUPS_ALONG_X", "1")
        op1 = bri.OverlapOp(L, W[bri.F64], kl_n=8, rho=1.0, tol=1e-12, nrhs=3)
        got, st = op1.apply(bd)
        torch.cuda.synchronize()
    finally:
        bri.set_stencil_cfg(L, bri.F64, 3, None)
    assert st.iters == st_ref.iters
    assert list(st.shift_iters) == list(st_ref.shift_iters)
    assert torch.equal(got, ref)
    Wo = oracle.links(L, U)
    g = bri.spinor_to_host(got)
    for c in range(3):
        want, _, _ = oracle.ov_apply(L, Wo, 1.0, 8, b[c], tol=1e-13)
        assert rel_l2(g[c], want) < 1e-10, c
