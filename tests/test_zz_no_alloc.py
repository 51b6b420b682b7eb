"""ov_apply_noalloc (the overlap apply for callers that cannot allocate: workspace in the
library's static device scratch, no pinned memory, no HIP graphs) against ov_apply through the
C ABI: two calls in a row, the second smaller, FP64 and mixed precision, each equal to ov_apply
and within 1e-10 of the oracle (eq. (def_over)); a problem larger than the scratch is refused
with BRI_ESCRATCH before anything runs."""

import ctypes

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu


def _noalloc(L, W, Wlo, prm, psi, out):
    lib = bri.load()
    g = bri._geom(L, 0, bri._clover_flag(W))
    st = bri._OvStats()
    rc = lib.ov_apply_noalloc(ctypes.byref(g), bri._dptr(W), None if Wlo is None else bri._dptr(Wlo),
                              ctypes.byref(prm), bri._dptr(psi), bri._dptr(out), int(psi.shape[0]),
                              ctypes.byref(st), bri._stream())
    torch.cuda.synchronize()
    return rc, st


@pytest.mark.parametrize("inner", [bri.F64, bri.F32])
def test_noalloc_matches_ov_apply_twice(inner):
    need_gpu()
    for L, n, nrhs, seed in (((8, 8, 8, 8), 16, 2, 1801), ((4, 4, 4, 4), 8, 1, 1802)):
        print(f"[noalloc] L={L} n={n} nrhs={nrhs} inner={inner}", flush=True)
        U = synth.smeared_links(L, 0.5, seed, 0.6, 1)
        Ud = bri.links_to_device(U)
        W = bri.build_links(L, Ud, bri.F64)
        Wlo = None if inner == bri.F64 else bri.build_links(L, Ud, inner)
        b = synth.gaussian_source(L, seed + 7, nrhs=nrhs)
        bd = bri.spinor_to_device(b)
        op = bri.OverlapOp(L, W, kl_n=n, tol=1e-12, Wlo=Wlo, inner=inner, nrhs=nrhs)
        ref, st_ref = op.apply(bd)
        out = torch.full_like(bd, float("nan"))
        rc, st = _noalloc(L, W, Wlo, op.params, bd, out)
        assert rc == bri.OK, bri.STATUS_NAMES.get(rc, rc)
        assert st.iters == st_ref.iters
        got, want = bri.spinor_to_host(out), bri.spinor_to_host(ref)
        Wo = oracle.links(L, U)
        for r in range(nrhs):
            assert rel_l2(got[r], want[r]) < 1e-14
            oref, _, _ = oracle.ov_apply(L, Wo, 1.0, n, b[r], tol=1e-13)
            assert rel_l2(got[r], oref) < 1e-10


def test_noalloc_refuses_a_problem_beyond_the_scratch():
    need_gpu()
    lib = bri.load()
    cap = lib.ov_noalloc_max_bytes()
    assert cap == 256 << 20
    L = (16, 16, 16, 16)
    V = int(np.prod(L))
    # FP64, 16 shifts, two right-hand sides: about 2 x 19 vectors of 12 V complex doubles > 256 MiB
    op_bytes = ctypes.c_size_t(0)
    prm = bri._OvParams(16, 1.0, 1e-12, 100, 0, 0, 0, 0, 0)
    g = bri._geom(L)
    assert lib.ov_apply(ctypes.byref(g), None, None, ctypes.byref(prm), None, None, 2, None, ctypes.byref(op_bytes),
                        None, None) == bri.OK
    assert op_bytes.value > cap
    W = torch.zeros((40, 3, 3, V), dtype=torch.complex128, device="cuda")
    b = torch.zeros((2, 4, 3, V), dtype=torch.complex128, device="cuda")
    out = torch.full_like(b, 7.0)
    rc, _ = _noalloc(L, W, None, prm, b, out)
    assert rc == bri.ESCRATCH
    assert bool((out == 7.0).all())  # nothing ran
