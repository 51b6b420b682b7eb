"""The deferred shift updates of ov_apply (y and the shifted directions carried as coefficients of
the residuals a window of iterations stores, written once per window) against the same solve with
the updates taken every iteration, which ov_apply_noalloc keeps, through the C ABI.  Both compute
the sums of the multi-shift recurrences (Sec. 3.3) in another order, so they agree to rounding:
the same iteration counts and outputs within 1e-13 relative in FP64.  With an FP32 phase the
per-iteration form rounds every p_sigma to FP32 at each iteration and the deferred form once per
window, so the two differ by FP32 rounding of the late updates, whose size is set by tol: there
they must agree within tol / 10.  Cases where windows end at
different points of the solve: right-hand sides that stop at different iterations (a Gaussian and
two point sources), the switch to the FP32 phase inside a window, the result-bound and App. B
stopping rules, the upper-diagonal rational, and an iteration cap that ends the solve inside a
window (BRI_ENOCONV, the last iterate in both).  The oracle checks one case at 1e-10."""

import ctypes

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu

L8 = (8, 8, 8, 8)


def _per_iteration(L, W, Wlo, prm, psi):
    """ov_apply_noalloc: the same solve with the shift updates of every iteration applied at once."""
    out = torch.full_like(psi, float("nan"))
    g = bri._geom(L, 0, bri._clover_flag(W))
    st = bri._OvStats()
    rc = bri.load().ov_apply_noalloc(ctypes.byref(g), bri._dptr(W), None if Wlo is None else bri._dptr(Wlo),
                                     ctypes.byref(prm), bri._dptr(psi), bri._dptr(out), int(psi.shape[0]),
                                     ctypes.byref(st), bri._stream())
    torch.cuda.synchronize()
    return rc, out, st


@pytest.fixture(scope="module")
def field8():
    U = synth.smeared_links(L8, 0.5, synth.LINK_SEED_BASE + 61, 0.6, 2)
    Ud = bri.links_to_device(U)
    b = np.concatenate([synth.gaussian_source(L8, synth.SOURCE_SEED_BASE + 61), synth.point_sources_12(L8)[[0, 7]]])
    return U, bri.build_links(L8, Ud, bri.F64), bri.build_links(L8, Ud, bri.F32), b


CASES = {
    "fp64": dict(tol=1e-12),
    "fp32_phase": dict(tol=1e-12, inner=bri.F32),
    "result_bound": dict(tol=1e-10, relax=bri.RELAX_BOUND),
    "result_bound_fp32": dict(tol=1e-10, relax=bri.RELAX_BOUND, inner=bri.F32),
    "upper_relaxed": dict(tol=1e-11, kind=bri.KL_UPPER, relax=bri.RELAX_OMEGA),
}


@pytest.mark.parametrize("case", list(CASES))
def test_deferred_matches_per_iteration(field8, case):
    need_gpu()
    U, W, W32, b = field8
    kw = dict(CASES[case])
    inner = kw.pop("inner", bri.F64)
    agree = 1e-13 if inner == bri.F64 else 0.1 * kw["tol"]
    Wlo = W32 if inner == bri.F32 else None
    print(f"[deferred] {case}", flush=True)
    bd = bri.spinor_to_device(b)
    op = bri.OverlapOp(L8, W, kl_n=16, rho=1.0, max_iter=3000, Wlo=Wlo, inner=inner, nrhs=3, **kw)
    got, st = op.apply(bd)
    rc, ref, st_ref = _per_iteration(L8, W, Wlo, op.params, bd)
    assert rc == bri.OK, bri.STATUS_NAMES.get(rc, rc)
    assert st.iters == st_ref.iters and st.refine == st_ref.refine
    assert list(st.shift_iters)[:16] == list(st_ref.shift_iters)[:16]
    g, r = bri.spinor_to_host(got), bri.spinor_to_host(ref)
    for c in range(3):
        assert rel_l2(g[c], r[c]) < agree, (case, c, rel_l2(g[c], r[c]))
    if case == "fp64":
        Wo = oracle.links(L8, U)
        for c in range(3):
            oref, _, _ = oracle.ov_apply(L8, Wo, 1.0, 16, b[c], tol=1e-13)
            assert rel_l2(g[c], oref) < 1e-10


@pytest.mark.parametrize("inner", [bri.F64, bri.F32])
def test_deferred_iteration_cap_inside_a_window(field8, inner):
    """max_iter = 11 ends the solve three iterations into the second window: both forms return
    BRI_ENOCONV with the same last iterate."""
    need_gpu()
    U, W, W32, b = field8
    Wlo = W32 if inner == bri.F32 else None
    bd = bri.spinor_to_device(b)
    op = bri.OverlapOp(L8, W, kl_n=16, rho=1.0, tol=1e-13, max_iter=11, Wlo=Wlo, inner=inner, nrhs=3)
    got, st = op.apply(bd, allow_noconv=True)
    assert st.status == bri.ENOCONV and st.iters == 11
    rc, ref, st_ref = _per_iteration(L8, W, Wlo, op.params, bd)
    assert rc == bri.ENOCONV and st_ref.iters == 11
    g, r = bri.spinor_to_host(got), bri.spinor_to_host(ref)
    for c in range(3):
        assert rel_l2(g[c], r[c]) < (1e-13 if inner == bri.F64 else 1e-12), (c, rel_l2(g[c], r[c]))
