"""Every launch configuration the autotuner may pick computes the same
operator: bri_apply / bri_apply_dag under each candidate tile, traversal and
work split are checked against the oracle (App. C.1 stencil), and the tuner
installs a configuration the solvers then use."""

import itertools

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu

L = (16, 8, 8, 6)


def _configs(nrhs):
    # (tile x, y, z, t, col_z, col_y); the last two: columns two tile rows wide (y fastest inside)
    trav = [(0, 0, 0, 0, 0, 0), (16, 4, 1, 1, 0, 0), (4, 4, 4, 1, 0, 0)]
    trav += [(tx, ty, 1, 1, cz, 0) for (tx, ty), cz in itertools.product([(8, 8), (16, 4)], [2, 4, 8])]
    trav += [(16, 4, 1, 1, cz, 2) for cz in (2, 8)]
    work = [(2, 0), (4, 0), (1, 0)] if nrhs == 1 else [(4, 0), (4, 1), (4, 2), (4, 3), (4, 4)]
    for t, w, xcd in itertools.product(trav, work, (0, 1)):
        yield bri.StencilCfg(t[0], t[1], t[2], t[3], t[4], w[0], w[1], xcd, 0, t[5])
    # the x-line kernel (tile_x = L_x) in y-blocked columns, one or several RHS per thread
    for cz, xcd, rpt in itertools.product((2, 4), (0, 1), (0,) if nrhs == 1 else (0, 2, 3)):
        yield bri.StencilCfg(16, 4, 1, 1, cz, 4, rpt, xcd, 2, 2)


@pytest.fixture(scope="module")
def setup():
    U = synth.random_links(L, 0.6, 4242)
    Wo = oracle.links(L, U)
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    return Wo, W


@pytest.mark.parametrize("nrhs", [1, 2, 5])
def test_every_config_matches_oracle(setup, nrhs):
    need_gpu()
    Wo, W = setup
    psi = synth.gaussian_source(L, 31 + nrhs, nrhs=nrhs)
    ref = oracle.dirac(L, Wo, -0.9, psi)
    ref_dag = oracle.dirac_adj(L, Wo, -0.9, psi)
    x = bri.spinor_to_device(psi)
    n = 0
    try:
        for cfg in _configs(nrhs):
            bri.set_stencil_cfg(L, bri.F64, nrhs, cfg)
            got = bri.spinor_to_host(bri.apply(L, W, bri.F64, -0.9, x))
            gotd = bri.spinor_to_host(bri.apply_dag(L, W, bri.F64, -0.9, x))
            for r in range(nrhs):
                assert rel_l2(got[r], ref[r]) < 1e-14, cfg.as_dict()
                assert rel_l2(gotd[r], ref_dag[r]) < 1e-14, cfg.as_dict()
            n += 1
    finally:
        bri.set_stencil_cfg(L, bri.F64, nrhs, None)
    assert n >= 20


def test_autotune_installs_and_solver_uses_it(setup):
    need_gpu()
    Wo, W = setup
    x = bri.spinor_to_device(synth.gaussian_source(L, 77))
    try:
        best, us = bri.autotune(L, W, bri.F64, x, reps=2)
        assert us > 0
        got = bri.get_stencil_cfg(L, bri.F64, 1)
        assert got.as_dict() == best.as_dict()
        op = bri.OverlapOp(L, W, kl_n=6, tol=1e-12)
        b = synth.gaussian_source(L, 78)
        out, _ = op.apply(bri.spinor_to_device(b))
        ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 6, b[0], tol=1e-13)
        assert rel_l2(bri.spinor_to_host(out)[0], ref) < 1e-10
    finally:
        bri.set_stencil_cfg(L, bri.F64, 1, None)


def test_invalid_config_rejected():
    need_gpu()
    with pytest.raises(bri.BriError):
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(5, 4, 1, 1, 0, 4, 0, 1))
    with pytest.raises(bri.BriError):
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(8, 8, 1, 1, 5, 4, 0, 1))
    # col_y must divide the tile rows along y (2 here) and needs the column traversal
    with pytest.raises(bri.BriError):
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 0, 3))
    with pytest.raises(bri.BriError):
        bri.set_stencil_cfg(L, bri.F64, 1, bri.StencilCfg(16, 4, 1, 1, 0, 4, 0, 1, 0, 2))
