"""GPU parity of ov_apply / ov_sign_apply (eq. (def_over) with the Kenney-Laub
rational of eq. (KLnn_parfrac)) against the oracle's per-shift CG evaluation
and the dense 4^4 eigendecomposition, plus error paths.

Tolerance: 1e-10 relative (L2) on the result, the accuracy the overlap apply
is asked to deliver; the solver runs at CG tolerance 1e-12.
"""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from oracle import dense as odense
from tests._gpu import field, need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _op(L, U, n, tol=1e-12, max_iter=2000, tbc=0, nrhs=1):
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=tbc)
    return bri.OverlapOp(L, W, kl_n=n, rho=1.0, tol=tol, max_iter=max_iter, tbc=tbc, nrhs=nrhs)


@pytest.mark.parametrize("kind", ["unit", "cfg1"])
@pytest.mark.parametrize("n", [8, 16])
def test_overlap_4_4_point_source(kind, n):
    need_gpu()
    L = (4, 4, 4, 4)
    U, Wo = field(L, kind)
    op = _op(L, U, n)
    b = synth.point_source(L)
    out, st = op.apply(bri.spinor_to_device(b))
    got = bri.spinor_to_host(out)[0]
    ref, it, rel = oracle.ov_apply(L, Wo, 1.0, n, b[0], tol=1e-13)
    assert rel_l2(got, ref) < TOL, (st.iters, st.shift_iters)
    assert st.iters > 0 and max(st.rel_resid) <= 1e-12
    s_out, _ = op.sign(bri.spinor_to_device(b))
    sref, _, _ = oracle.sign_apply(L, Wo, 1.0, n, b[0], tol=1e-13)
    assert rel_l2(bri.spinor_to_host(s_out)[0], sref) < TOL


@pytest.mark.parametrize("kind", [bri.KL_DIAG, bri.KL_UPPER])
def test_overlap_maximum_order(kind):
    """Every one of the BRI_MAX_SHIFTS shifts runs (one scalar thread per shift in the solver)."""
    need_gpu()
    L = (4, 4, 4, 4)
    n = bri.MAX_SHIFTS
    U, Wo = field(L, "cfg1")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    op = bri.OverlapOp(L, W, kl_n=n, rho=1.0, tol=1e-12, max_iter=2000, kind=kind)
    g = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 7)
    out, st = op.apply(bri.spinor_to_device(g))
    kname = "diag" if kind == bri.KL_DIAG else "upper"
    ref, _, _ = oracle.ov_apply(L, Wo, 1.0, n, g[0], tol=1e-13, kind=kname)
    assert rel_l2(bri.spinor_to_host(out)[0], ref) < TOL
    assert len(st.shift_iters) == n and all(0 < k <= st.iters for k in st.shift_iters)
    assert max(st.rel_resid) <= 1e-12
    # the smallest shift is the base system and converges last
    assert st.shift_iters[0] == st.iters


def test_overlap_against_dense_eigendecomposition():
    need_gpu()
    L = (4, 4, 4, 4)
    U, Wo = field(L, "cfg1")
    dov = odense.DenseOverlap(oracle.dense_matrix(L, Wo, -1.0), 256, 1.0)
    op = _op(L, U, 8, nrhs=2)
    g = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 1, nrhs=2)
    out, _ = op.apply(bri.spinor_to_device(g))
    got = bri.spinor_to_host(out)
    for r in range(2):
        want = dov.ov_apply(8, g[r].reshape(-1)).reshape(g[r].shape)
        assert rel_l2(got[r], want) < TOL
    # and the sign function within the [8/8] approximation bound of this spectrum
    s_out, _ = op.sign(bri.spinor_to_device(g[:1]))
    exact = dov.sign_exact_apply(g[0].reshape(-1)).reshape(g[0].shape)
    assert np.linalg.norm(bri.spinor_to_host(s_out)[0] - exact) <= dov.sign_bound(8) * 1.01 + 1e-11


@pytest.mark.parametrize("L,tbc", [((4, 8, 4, 6), 0), ((4, 4, 4, 8), 1), ((16, 4, 1, 1), 1), ((2, 2, 2, 8), 0)])
def test_overlap_non_cubic(L, tbc):
    need_gpu()
    U = synth.random_links(L, 0.4, 77)
    Wo = oracle.links(L, U, tbc=tbc)
    op = _op(L, U, 6, tbc=tbc)
    b = synth.gaussian_source(L, 78)
    out, _ = op.apply(bri.spinor_to_device(b))
    ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 6, b[0], tol=1e-13)
    assert rel_l2(bri.spinor_to_host(out)[0], ref) < TOL


def test_sign_squared_at_bench_size():
    """16^4 smeared field, [16/16]: sign(H)^2 b = b and the Ginsparg-Wilson
    identity D g5 + g5 D = D g5 D / rho (eq. (ginswils_one)) hold to the
    rational approximation's accuracy."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, _ = field(L, "cfg2")
    op = _op(L, U, 16)
    b = bri.spinor_to_device(synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 2))
    s1, st1 = op.sign(b)
    s2, _ = op.sign(s1)
    assert float(torch.linalg.vector_norm(s2 - b) / torch.linalg.vector_norm(b)) < 1e-9
    g5 = torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=torch.float64, device=b.device).view(1, 4, 1, 1)
    Db, _ = op.apply(b)
    Dg5b, _ = op.apply(b * g5)
    Dg5Db, _ = op.apply(Db * g5)
    gw = Dg5b + g5 * Db - Dg5Db
    assert float(torch.linalg.vector_norm(gw) / torch.linalg.vector_norm(b)) < 1e-9
    assert 10 < st1.iters < 500


def test_noconv_status_and_stats():
    need_gpu()
    L = (4, 4, 4, 4)
    U, _ = field(L, "cfg1")
    op = _op(L, U, 8, max_iter=2)
    out, st = op.apply(bri.spinor_to_device(synth.point_source(L)), allow_noconv=True)
    assert st.status == bri.ENOCONV and st.iters == 2
    with pytest.raises(bri.BriError):
        op.apply(bri.spinor_to_device(synth.point_source(L)))


def test_nan_input_status():
    need_gpu()
    L = (4, 4, 4, 4)
    U, _ = field(L, "cfg1")
    op = _op(L, U, 8)
    b = synth.point_source(L)
    b[0, 3, 1, 2] = np.nan
    with pytest.raises(bri.BriError) as e:
        op.apply(bri.spinor_to_device(b))
    assert e.value.status == bri.ENAN


def test_zero_source_and_repeatability():
    need_gpu()
    L = (4, 8, 4, 6)
    U, _ = field(L, "rough")
    op = _op(L, U, 8)
    z, st = op.apply(bri.spinor_to_device(np.zeros((1, 768, 4, 3), dtype=np.complex128)))
    assert float(torch.abs(z).max()) == 0.0 and st.iters == 0
    b = bri.spinor_to_device(synth.gaussian_source(L, 5))
    a1, _ = op.apply(b)
    a2, _ = op.apply(b)
    assert torch.equal(a1, a2)
