"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/brillouin.h declares, computes the Kenney-Laub
coefficients of eq. (KLnn_parfrac) on the host, sizes its workspace and rejects
bad arguments before launching anything."""

import ctypes
import os
import re

import mpmath as mp
import pytest

import paper_1701_00726_amd as bri
from oracle import kl
from tests.conftest import ROOT


def _declared():
    txt = open(os.path.join(ROOT, "include", "brillouin.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_exports_every_declared_symbol():
    lib = bri.load()
    names = _declared()
    assert set(names) == set(bri.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("n", [1, 2, 4, 8, 13, 16, 32])
def test_host_kl_coefficients_match_oracle(n):
    c0, om, sg = bri.kl_coeffs(n)
    rc0, rom, rsg = kl.kl_diag_coeffs(n)
    assert abs(c0 - float(rc0)) == 0
    assert sg == sorted(sg)
    for a, b in zip(om, rom):
        assert abs(mp.mpf(a) - b) <= 6e-16 * abs(b)
    for a, b in zip(sg, rsg):
        assert abs(mp.mpf(a) - b) <= 6e-16 * abs(b)


def _ov_query(L, **kw):
    g = bri._geom(L)
    prm = bri._OvParams(kw.get("kl_n", 8), kw.get("rho", 1.0), kw.get("tol", 1e-10), kw.get("max_iter", 100),
                        kw.get("inner", 0), kw.get("max_refine", 0))
    nb = ctypes.c_size_t(0)
    st = bri.load().ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb),
                             None, None)
    return st, nb.value


def test_workspace_query():
    st, nbytes = _ov_query((16, 16, 16, 16), kl_n=16)
    V = 16**4
    assert st == bri.OK
    # r, p, t, y, 15 shifted directions, the base direction at the window's start and 8 stored
    # residuals of 12 V complex doubles, plus small state
    assert 28 * 12 * V * 16 <= nbytes < 28 * 12 * V * 16 + (1 << 20)


@pytest.mark.parametrize(
    "L,kw",
    [
        ((16, 16, 16, 16), dict(kl_n=0)),
        ((16, 16, 16, 16), dict(kl_n=33)),
        ((16, 16, 16, 16), dict(rho=2.0)),
        ((16, 16, 16, 16), dict(rho=0.0)),
        ((16, 16, 16, 16), dict(tol=0.0)),
        ((16, 16, 16, 16), dict(max_iter=0)),
        ((16, 16, 16, 16), dict(inner=7)),
        ((3, 3, 3, 3), dict()),
        ((0, 4, 4, 4), dict()),
    ],
)
def test_invalid_arguments(L, kw):
    st, _ = _ov_query(L, **kw)
    assert st == bri.EINVAL


def test_invalid_stencil_arguments():
    lib = bri.load()
    g = bri._geom((5, 5, 4, 4))  # V = 400 is not a whole number of 64-site tiles
    assert lib.bri_apply(ctypes.byref(g), ctypes.c_void_p(16), 0, -1.0, ctypes.c_void_p(16), ctypes.c_void_p(32), 1,
                         None) == bri.EINVAL
    g = bri._geom((4, 4, 4, 4))
    assert lib.bri_apply(ctypes.byref(g), None, 0, -1.0, ctypes.c_void_p(16), ctypes.c_void_p(32), 1, None) == bri.EINVAL
    assert lib.bri_apply_dag(ctypes.byref(g), ctypes.c_void_p(16), 9, -1.0, ctypes.c_void_p(16), ctypes.c_void_p(32),
                             1, None) == bri.EINVAL
    assert lib.bri_build_links(None, ctypes.c_void_p(16), ctypes.c_void_p(16), 0, None) == bri.EINVAL
    assert lib.bri_build_links(ctypes.byref(g), ctypes.c_void_p(16), ctypes.c_void_p(16), 5, None) == bri.EINVAL
    g.tbc = 2
    assert lib.bri_build_links(ctypes.byref(g), ctypes.c_void_p(16), ctypes.c_void_p(16), 0, None) == bri.EINVAL
    g.tbc = 0
    P = ctypes.c_void_p
    assert lib.bri_round_links(None, P(1 << 24), P(1 << 26), 1, None) == bri.EINVAL
    assert lib.bri_round_links(ctypes.byref(g), None, P(1 << 26), 1, None) == bri.EINVAL
    assert lib.bri_round_links(ctypes.byref(g), P(1 << 24), None, 2, None) == bri.EINVAL
    for prec in (0, 3, -1):  # FP64 is the source precision, not a target
        assert lib.bri_round_links(ctypes.byref(g), P(1 << 24), P(1 << 26), prec, None) == bri.EINVAL
    # the rounded array written over the FP64 one
    assert lib.bri_round_links(ctypes.byref(g), P(1 << 24), P((1 << 24) + 64), 1, None) == bri.EINVAL
    assert lib.bri_round_links(ctypes.byref(g), P(1 << 24), P((1 << 24) - 4096), 2, None) == bri.EINVAL


def test_stencil_config_col_y_validated_and_kept():
    """Host-side validation of the y-blocked column traversal (no launch): col_y must divide the
    tile rows along y and needs col_z > 0; an accepted configuration reads back unchanged."""
    L = (16, 16, 8, 8)  # 16 x 4 tiles: four tile rows along y
    try:
        good = bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 2, 4)
        bri.set_stencil_cfg(L, bri.F64, 1, good)
        assert bri.get_stencil_cfg(L, bri.F64, 1).as_dict() == good.as_dict()
        for bad in (bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 0, 3),   # 3 does not divide 4 rows
                    bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 0, 8),   # wider than the lattice
                    bri.StencilCfg(16, 4, 1, 1, 0, 4, 0, 1, 0, 2),   # lexicographic tiles
                    bri.StencilCfg(16, 4, 1, 1, 2, 4, 0, 1, 0, -1)):
            with pytest.raises(bri.BriError):
                bri.set_stencil_cfg(L, bri.F64, 1, bad)
    finally:
        bri.set_stencil_cfg(L, bri.F64, 1, None)


@pytest.mark.parametrize("L", [(32, 32, 32, 64), (16, 16, 16, 16), (24, 24, 24, 48), (64, 8, 16, 16),
                               (16, 32, 8, 32), (8, 8, 8, 8)])
def test_default_configs_are_valid(L):
    """Host-side: the default launch configuration of every precision and batch size is one the
    validation accepts (tile, column width and depth dividing the lattice) and reads back unchanged
    when installed."""
    for prec in (bri.F64, bri.F32, bri.F32_BF16W):
        for nrhs in (1, 2, 3, 12):
            d = bri.get_stencil_cfg(L, prec, nrhs)
            try:
                bri.set_stencil_cfg(L, prec, nrhs, d)
                assert bri.get_stencil_cfg(L, prec, nrhs).as_dict() == d.as_dict()
            finally:
                bri.set_stencil_cfg(L, prec, nrhs, None)
    if L == (32, 32, 32, 64):  # whole-line tiles in y-blocked columns on the benchmark lattice
        d1 = bri.get_stencil_cfg(L, bri.F64, 1)
        assert (d1.tile_x, d1.tile_y, d1.col_z, d1.col_y, d1.variant) == (32, 2, 4, 8, 2)
        assert bri.get_stencil_cfg(L, bri.F32, 1).col_y == 16
        assert bri.get_stencil_cfg(L, bri.F32, 12).col_y == 2


def test_gradient_workspace_and_invalid_arguments():
    lib = bri.load()
    L = (8, 8, 8, 8)
    V = 8**4
    g = bri._geom(L)
    nb = ctypes.c_size_t(0)
    w = (ctypes.c_double * 1)(1.0)
    assert lib.bri_link_grad(ctypes.byref(g), None, None, 1, w, None, None, None, None, None, ctypes.byref(nb),
                             None) == bri.OK
    assert nb.value == 81 * 9 * V * 16  # one 3x3 complex double per site and displacement
    for npairs in (0, bri.MAX_PAIRS + 1):
        assert lib.bri_link_grad(ctypes.byref(g), None, None, npairs, w, None, None, None, None, None,
                                 ctypes.byref(nb), None) == bri.EINVAL
    # neither F nor GU requested: rejected before any launch
    nb2 = ctypes.c_size_t(1 << 40)
    assert lib.bri_link_grad(ctypes.byref(g), ctypes.c_void_p(16), ctypes.c_void_p(16), 1, w, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), None, None, ctypes.c_void_p(16), ctypes.byref(nb2),
                             None) == bri.EINVAL
    prm = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0)
    assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None,
                             None, ctypes.byref(nb), None, None) == bri.OK
    # G, the 2n applied shift solutions, [psi | X^dag chi], y, and the two-column multi-shift
    # (r, p, t: 3 x 2 columns; x: 8 x 2; shifted directions: 7 x 2; the window's base direction
    # and 8 stored residuals: 9 x 2)
    vec = 12 * V * 16
    assert 81 * 9 * V * 16 + vec * (16 + 2 + 1 + 6 + 16 + 14 + 18) <= nb.value
    assert nb.value < 81 * 9 * V * 16 + vec * (16 + 2 + 1 + 6 + 16 + 14 + 18) + (1 << 20)
    for bad in (bri._OvParams(8, 1.0, 1e-10, 100, 7, 0), bri._OvParams(0, 1.0, 1e-10, 100, 0, 0),
                bri._OvParams(8, 2.0, 1e-10, 100, 0, 0), bri._OvParams(8, 1.0, 1e-10, 100, 1, 101)):
        assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(bad), None, None, None, None, None,
                                 None, ctypes.byref(nb), None, None) == bri.EINVAL
    # a low-precision inner solve adds the FP32 vectors of its late iterations: larger
    lo = bri._OvParams(8, 1.0, 1e-10, 100, 1, 10)
    nb_lo = ctypes.c_size_t(0)
    assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(lo), None, None, None, None, None, None,
                             ctypes.byref(nb_lo), None, None) == bri.OK
    assert nb_lo.value > nb.value
    # recomputed shift solutions, two shifts per solve: G, the 4 applied solutions, [psi | X^dag chi], y
    # and a two-column two-shift solve (r, p, t: 3 x 2; x: 2 x 2; shifted directions: 1 x 2)
    rcp = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0, 0, 0, 0, 2)
    nb_r = ctypes.c_size_t(0)
    assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(rcp), None, None, None, None, None, None,
                             ctypes.byref(nb_r), None, None) == bri.OK
    assert 81 * 9 * V * 16 + vec * (4 + 2 + 1 + 6 + 4 + 2) <= nb_r.value < nb.value
    for m in (-1, bri.MAX_SHIFTS + 1):
        bad = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0, 0, 0, 0, m)
        assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(bad), None, None, None, None, None,
                                 None, ctypes.byref(nb), None, None) == bri.EINVAL


def test_solver_graph_switch_rejects_other_values():
    lib = bri.load()
    assert lib.bri_set_solver_graphs(2) == bri.EINVAL
    assert lib.bri_set_solver_graphs(-1) == bri.EINVAL


def test_massive_solve_workspace_and_invalid_args():
    lib = bri.load()
    L = (8, 8, 8, 8)
    V = 8**4
    g = bri._geom(L)
    prm = bri._OvParams(8, 1.0, 1e-12, 200, 0, 0)
    st, ov_bytes = _ov_query(L, kl_n=8, tol=1e-12, max_iter=200)
    assert st == bri.OK
    nb = ctypes.c_size_t(0)
    mp_ = bri._MassParams(0.1, 1, 1e-10, 100)
    assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_), 0, None, None, None, 1, None,
                        ctypes.byref(nb), None, None) == bri.OK
    # the ov_apply workspace plus bt and eight BiCGstab vectors (r, r0, p, v, s, t, K p, K s) and
    # dot partials
    vec = 12 * V * 16
    assert ov_bytes + 9 * vec <= nb.value < ov_bytes + 9 * vec + (1 << 16)
    for bad in (bri._MassParams(-0.1, 1, 1e-10, 100), bri._MassParams(2.0, 1, 1e-10, 100),
                bri._MassParams(0.1, 2, 1e-10, 100), bri._MassParams(0.1, 1, 0.0, 100),
                bri._MassParams(0.1, 0, 1e-10, 0)):
        assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(bad), 0, None, None, None, 1,
                            None, ctypes.byref(nb), None, None) == bri.EINVAL
    # bad inner parameters are rejected through the ov_apply query
    badp = bri._OvParams(0, 1.0, 1e-12, 200, 0, 0)
    assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(badp), ctypes.byref(mp_), 0, None, None, None, 1, None,
                        ctypes.byref(nb), None, None) == bri.EINVAL
    # a workspace that is too small, or in == out, is rejected before any launch
    small = ctypes.c_size_t(nb.value - 1)
    p = ctypes.c_void_p(256)
    assert lib.ov_solve(ctypes.byref(g), p, None, ctypes.byref(prm), ctypes.byref(mp_), 0, None, p, ctypes.c_void_p(512),
                        1, p, ctypes.byref(small), None, None) == bri.EINVAL
    full = ctypes.c_size_t(nb.value)
    assert lib.ov_solve(ctypes.byref(g), p, None, ctypes.byref(prm), ctypes.byref(mp_), 0, None, p, p, 1, p,
                        ctypes.byref(full), None, None) == bri.EINVAL


def test_cascade_levels_validated():
    lib = bri.load()
    L = (8, 8, 8, 8)
    V = 8**4
    vec = 12 * V * 16
    g = bri._geom(L)
    prm = bri._OvParams(4, 1.0, 1e-12, 200, 0, 0)
    mp_ = bri._MassParams(0.03, 1, 1e-9, 100)

    def query(levels, n=None):
        arr = (bri._Level * max(len(levels), 1))(*levels)
        nb = ctypes.c_size_t(0)
        st = lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_),
                          len(levels) if n is None else n, arr, None, None, 1, None, ctypes.byref(nb), None, None)
        return st, nb.value

    st0, nb0 = query([])
    assert st0 == bri.OK
    # the paper's two-level cascade for f_{4,4}: n = 1, then the Brillouin operator
    st2, nb2 = query([bri._Level(1, 0.1, 20, 1e-6, 0), bri._Level(0, 0.1, 20, 0.0, 0)])
    # eight BiCGstab vectors per level, and two for the compacted columns of the FP64 kernel level
    assert st2 == bri.OK and nb2 == nb0 + (2 * 8 + 2) * vec
    bads = [
        [bri._Level(0, 0.1, 20, 0.0, 0), bri._Level(1, 0.1, 20, 1e-6, 0)],  # Brillouin not last
        [bri._Level(1, 0.0, 20, 1e-6, 0)],                                 # tol <= 0
        [bri._Level(1, 0.1, 0, 1e-6, 0)],                                  # no iterations
        [bri._Level(1, 0.1, 20, 0.0, 0)],                                  # multi-shift tol <= 0
        [bri._Level(bri.MAX_SHIFTS + 1, 0.1, 20, 1e-6, 0)],                # order too large
        [bri._Level(-1, 0.1, 20, 1e-6, 0)],
        [bri._Level(1, 0.1, 20, 1e-6, 9)],                                 # unknown precision
    ]
    for lv in bads:
        assert query(lv)[0] == bri.EINVAL, lv
    assert query([bri._Level(1, 0.1, 20, 1e-6, 0)] * 5)[0] == bri.EINVAL  # more than BRI_MAX_LEVELS
    assert query([], n=1)[0] == bri.EINVAL  # a level count without levels
    # a low-precision level needs Wlo: rejected at the call, before any launch
    arr = (bri._Level * 1)(bri._Level(1, 0.1, 20, 1e-5, 1))
    nb = ctypes.c_size_t(0)
    assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_), 1, arr, None, None, 1,
                        None, ctypes.byref(nb), None, None) == bri.OK
    p = ctypes.c_void_p(256)
    assert lib.ov_solve(ctypes.byref(g), p, None, ctypes.byref(prm), ctypes.byref(mp_), 1, arr, p,
                        ctypes.c_void_p(512), 1, p, ctypes.byref(nb), None, None) == bri.EINVAL


@pytest.mark.parametrize("n", [1, 2, 3, 8, 16, 32])
def test_host_upper_diagonal_coefficients_match_oracle(n):
    om, sg = bri.kl_upper_coeffs(n)
    rom, rsg = kl.kl_upper_coeffs(n)
    assert sg == sorted(sg)
    for a, b in zip(om, rom):
        assert abs(mp.mpf(a) - b) <= 6e-16 * abs(b)
    for a, b in zip(sg, rsg):
        assert abs(mp.mpf(a) - b) <= 6e-16 * abs(b)


def test_kind_and_relax_validated():
    assert _ov_query((8, 8, 8, 8))[0] == bri.OK
    lib = bri.load()
    g = bri._geom((8, 8, 8, 8))
    nb = ctypes.c_size_t(0)
    for kind, relax, want in ((1, 0, bri.OK), (0, 1, bri.OK), (1, 1, bri.OK), (2, 0, bri.EINVAL),
                              (-1, 0, bri.EINVAL), (0, 3, bri.EINVAL), (0, -1, bri.EINVAL)):
        prm = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0, kind, relax)
        assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb),
                            None, None) == want, (kind, relax)
        assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None,
                                 None, ctypes.byref(nb), None, None) == want, (kind, relax)
    # the result bound: the applies accept it, the gradient does not
    for kind in (0, 1):
        prm = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0, kind, bri.RELAX_BOUND)
        assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb),
                            None, None) == bri.OK
        assert lib.ov_sign_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None,
                                 ctypes.byref(nb), None, None) == bri.OK
        assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None,
                                 None, ctypes.byref(nb), None, None) == bri.EINVAL
    om = (ctypes.c_double * 1)()
    assert lib.bri_kl_upper_coeffs(0, om, om) == bri.EINVAL
    assert lib.bri_kl_upper_coeffs(bri.MAX_SHIFTS + 1, om, om) == bri.EINVAL


def test_kernel_selector_validated():
    lib = bri.load()
    g = bri._geom((8, 8, 8, 8))
    nb = ctypes.c_size_t(0)
    for kernel, want_apply, want_grad in ((0, bri.OK, bri.OK), (1, bri.OK, bri.OK), (2, bri.EINVAL, bri.EINVAL)):
        prm = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0, 0, 0, kernel)
        assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb),
                            None, None) == want_apply
        assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None,
                                 None, ctypes.byref(nb), None, None) == want_grad
    # the Wilson applies validate like bri_apply before launching anything
    assert lib.wil_apply(ctypes.byref(g), None, 0, 0.0, None, None, 1, None) == bri.EINVAL
    assert lib.wil_apply_dag(ctypes.byref(g), ctypes.c_void_p(256), 7, 0.0, ctypes.c_void_p(256),
                             ctypes.c_void_p(512), 1, None) == bri.EINVAL


def test_clover_geometry_validated():
    lib = bri.load()
    nb = ctypes.c_size_t(0)
    g = bri._geom((8, 8, 8, 8), 0, float("nan"))
    prm = bri._OvParams(8, 1.0, 1e-10, 100, 0, 0)
    assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb), None,
                        None) == bri.EINVAL
    g = bri._geom((8, 8, 8, 8), 0, 1.0)
    assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb), None,
                        None) == bri.OK
    # the force does not differentiate the clover term: rejected before any launch
    assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None, None,
                             ctypes.byref(nb), None, None) == bri.EINVAL
    w = (ctypes.c_double * 1)(1.0)
    assert lib.bri_link_grad(ctypes.byref(g), None, None, 1, w, None, None, None, None, None, ctypes.byref(nb),
                             None) == bri.EINVAL
    # site indices are 32-bit: V = 2^31 is refused, V = 2^31 - 2^24 is sized (query only)
    big = bri._geom((4096, 4096, 128, 1), 0, 1.0)
    assert lib.bri_build_links(ctypes.byref(big), ctypes.c_void_p(256), ctypes.c_void_p(256), 0, None) == bri.EINVAL
    prm0 = bri._OvParams(4, 1.0, 1e-12, 200, 0, 0)
    for L, want in (((4096, 4096, 128, 1), bri.EINVAL), ((4096, 4096, 127, 1), bri.OK)):
        nb = ctypes.c_size_t(0)
        assert lib.ov_apply(ctypes.byref(bri._geom(L)), None, None, ctypes.byref(prm0), None, None, 1, None,
                            ctypes.byref(nb), None, None) == want, L
        if want == bri.OK:
            assert nb.value >= 7 * 12 * 16 * (4096 * 4096 * 127)  # r, p, t, y and 3 shifted directions


def test_massive_solve_nrhs_validated():
    lib = bri.load()
    g = bri._geom((8, 8, 8, 8))
    prm = bri._OvParams(4, 1.0, 1e-12, 200, 0, 0)
    mp_ = bri._MassParams(0.1, 1, 1e-10, 100)
    sizes = []
    for nrhs, want in ((0, bri.EINVAL), (1, bri.OK), (4, bri.OK), (bri.MAX_SOLVE_RHS, bri.OK),
                       (bri.MAX_SOLVE_RHS + 1, bri.EINVAL)):
        nb = ctypes.c_size_t(0)
        assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_), 0, None, None, None,
                            nrhs, None, ctypes.byref(nb), None, None) == want, nrhs
        if want == bri.OK:
            sizes.append((nrhs, nb.value))
    # nine vectors per column beyond the batched ov_apply workspace
    vec = 12 * 8**4 * 16
    for nrhs, nbytes in sizes:
        _, ovb = _ov_query((8, 8, 8, 8), kl_n=4, tol=1e-12, max_iter=200)
        assert nbytes >= 9 * vec * nrhs


def test_cascade_low_precision_levels_must_agree():
    lib = bri.load()
    g = bri._geom((8, 8, 8, 8))
    prm = bri._OvParams(4, 1.0, 1e-12, 200, 0, 0)
    mp_ = bri._MassParams(0.03, 1, 1e-9, 100)

    def query(levels):
        arr = (bri._Level * len(levels))(*levels)
        nb = ctypes.c_size_t(0)
        return lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_), len(levels), arr,
                            None, None, 1, None, ctypes.byref(nb), None, None), nb.value

    st64, nb64 = query([bri._Level(1, 0.1, 20, 1e-6, 0), bri._Level(0, 0.1, 20, 0.0, 0)])
    st32, nb32 = query([bri._Level(1, 0.1, 20, 1e-6, 0), bri._Level(0, 0.1, 20, 0.0, 1)])
    assert st64 == bri.OK and st32 == bri.OK
    # the narrowed kernel level keeps its two work vectors in complex float instead of double
    assert nb64 - nb32 == 2 * 12 * 8**4 * 8
    # one Wlo array: FP32 and bfloat16 levels cannot be mixed
    assert query([bri._Level(1, 0.1, 20, 1e-5, 1), bri._Level(0, 0.1, 20, 0.0, 2)])[0] == bri.EINVAL
    assert query([bri._Level(1, 0.1, 20, 1e-5, 2), bri._Level(0, 0.1, 20, 0.0, 2)])[0] == bri.OK


def test_binding_rejects_mismatched_outputs():
    """A caller-supplied output of the wrong dtype or shape is refused before any launch, since
    the kernels write the full size of the expected layout into it."""
    import torch

    L = (4, 4, 4, 4)
    V = 256
    psi = torch.zeros((1, 4, 3, V), dtype=torch.complex128)
    W = torch.zeros((40, 3, 3, V), dtype=torch.complex128)
    U = torch.zeros((4, 3, 3, V), dtype=torch.complex128)
    for bad in (torch.zeros((1, 4, 3, V), dtype=torch.complex64), torch.zeros((1, 4, 3, V - 1), dtype=torch.complex128)):
        with pytest.raises(ValueError, match="out must be"):
            bri.apply(L, W, bri.F64, -1.0, psi, out=bad)
    with pytest.raises(ValueError, match="out must be"):
        bri.build_links(L, U, bri.F64, out=torch.zeros((40, 3, 3, V), dtype=torch.complex64))
    with pytest.raises(ValueError, match="out must be"):
        bri.build_links(L, U, bri.F32, out=torch.zeros((40, 3, 3, V), dtype=torch.complex128))
    op = bri.OverlapOp(L, W, kl_n=4)
    with pytest.raises(ValueError, match="out must be"):
        op.apply(psi, out=torch.zeros((1, 4, 3, V), dtype=torch.complex64))


def test_aliased_arguments_rejected():
    """in / out (and the workspace) must not overlap: the stencil reads neighbours of in while it
    writes out, and the solvers keep vectors in the workspace.  Refused before any launch."""
    lib = bri.load()
    g = bri._geom((4, 4, 4, 4))
    sb = 12 * 256 * 16  # one complex-double spinor
    base = 1 << 20
    for off in (0, 16, sb - 16):  # identical, shifted by one entry, overlapping tails
        assert lib.bri_apply(ctypes.byref(g), ctypes.c_void_p(base), 0, -1.0, ctypes.c_void_p(base),
                             ctypes.c_void_p(base + off), 1, None) == bri.EINVAL, off
        assert lib.wil_apply_dag(ctypes.byref(g), ctypes.c_void_p(base), 0, -1.0, ctypes.c_void_p(base + off),
                                 ctypes.c_void_p(base), 1, None) == bri.EINVAL, off
    prm = bri._OvParams(4, 1.0, 1e-12, 200, 0, 0)
    nb = ctypes.c_size_t(0)
    assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 1, None, ctypes.byref(nb),
                        None, None) == bri.OK
    work = base + 64 * sb
    for inp, out in ((base, base), (base, base + sb // 2), (base, work + 256), (work, base)):
        wb = ctypes.c_size_t(nb.value)
        for fn in (lib.ov_apply, lib.ov_sign_apply):
            assert fn(ctypes.byref(g), ctypes.c_void_p(base + 32 * sb), None, ctypes.byref(prm), ctypes.c_void_p(inp),
                      ctypes.c_void_p(out), 1, ctypes.c_void_p(work), ctypes.byref(wb), None, None) == bri.EINVAL
    mp_ = bri._MassParams(0.1, 1, 1e-10, 100)
    sz = ctypes.c_size_t(0)
    assert lib.ov_solve(ctypes.byref(g), None, None, ctypes.byref(prm), ctypes.byref(mp_), 0, None, None, None, 1,
                        None, ctypes.byref(sz), None, None) == bri.OK
    for inp, out in ((base, base + 16), (base, work + 256)):
        wb = ctypes.c_size_t(sz.value)
        assert lib.ov_solve(ctypes.byref(g), ctypes.c_void_p(base + 32 * sb), None, ctypes.byref(prm),
                            ctypes.byref(mp_), 0, None, ctypes.c_void_p(inp), ctypes.c_void_p(out), 1,
                            ctypes.c_void_p(work), ctypes.byref(wb), None, None) == bri.EINVAL


def test_aliased_link_and_gradient_arguments_rejected():
    """The link build and the gradients refuse outputs or workspace that alias an input (or each
    other); all refused before any launch."""
    lib = bri.load()
    L = (4, 4, 4, 4)
    V = 256
    g = bri._geom(L)
    P = ctypes.c_void_p
    U, Wl = 1 << 24, 1 << 26  # disjoint stand-in addresses, never dereferenced
    # W written over U
    assert lib.bri_build_links(ctypes.byref(g), P(U), P(U + 64), 0, None) == bri.EINVAL
    assert lib.bri_build_links(ctypes.byref(g), P(U), P(U - 1000), 2, None) == bri.EINVAL
    # link force: F over u, GU over W, work over v, F over GU
    w = (ctypes.c_double * 1)(1.0)
    nb = ctypes.c_size_t(0)
    assert lib.bri_link_grad(ctypes.byref(g), None, None, 1, w, None, None, None, None, None, ctypes.byref(nb),
                             None) == bri.OK
    u, v, F, GU, work = 1 << 28, (1 << 28) + (1 << 22), 1 << 30, (1 << 30) + (1 << 22), 1 << 32
    for args in ((u, v, u + 16, None, work), (u, v, None, Wl, work), (u, v, F, None, v), (u, v, F, F + 8, work)):
        wb = ctypes.c_size_t(nb.value)
        assert lib.bri_link_grad(ctypes.byref(g), P(U), P(Wl), 1, w, P(args[0]), P(args[1]),
                                 P(args[2]) if args[2] else None, P(args[3]) if args[3] else None, P(args[4]),
                                 ctypes.byref(wb), None) == bri.EINVAL, args
    # overlap gradient: D_ov^dag chi written over chi, F over psi, work over U
    prm = bri._OvParams(4, 1.0, 1e-10, 100, 0, 0)
    nbg = ctypes.c_size_t(0)
    assert lib.ov_apply_grad(ctypes.byref(g), None, None, None, ctypes.byref(prm), None, None, None, None, None,
                             None, ctypes.byref(nbg), None, None) == bri.OK
    chi, psi, gpsi = 1 << 28, (1 << 28) + (1 << 22), (1 << 28) + (2 << 22)
    for c, p, f, gp, wk in ((chi, psi, F, chi, work), (chi, psi, psi, gpsi, work), (chi, psi, F, gpsi, U)):
        wb = ctypes.c_size_t(nbg.value)
        assert lib.ov_apply_grad(ctypes.byref(g), P(U), P(Wl), None, ctypes.byref(prm), P(c), P(p), P(f), None,
                                 P(gp), P(wk), ctypes.byref(wb), None, None) == bri.EINVAL
