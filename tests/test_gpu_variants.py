"""GPU parity of the sign-approximation variants (Sec. 3.3, App. B) through the C ABI:

  * the first upper diagonal g_{2n} (ov_params.kind = BRI_KL_UPPER) in ov_apply, ov_sign_apply
    and ov_apply_grad against the oracle's per-shift evaluation with the same coefficients
    (result tolerance 1e-10 relative, force 1e-9 of max|F|, as for the diagonal member);
  * relaxed per-shift stopping (ov_params.relax): every shift meets tol * omega_max / omega_i,
    the multi-shift stops no later than the strict one, and the result stays within the error
    bound its residuals imply, at 4^4 (against the dense exact rational) and at 16^4 (against
    the strict apply);
  * the result bound (relax = RELAX_BOUND): the reported residuals satisfy
    sum_i omega_i |r_i| / (2 sqrt(sigma_i)) <= tol, and the sign function lies within tol |b| of
    the dense exact rational at 4^4 (FP64 single source and batch; the FP32 low-precision phase
    within 2 tol |b|), and the 16^4 apply within rho tol |b| of the strict one, in fewer
    iterations.
"""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from oracle import dense as odense
from tests._gpu import field, need_gpu, rel_l2, torch
from tests.test_gpu_grad import _dev, _force_host, _rand_spinor

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)
TOL = 1e-10


def _op(L, U, n, tbc=0, **kw):
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=tbc)
    kw.setdefault("tol", 1e-12)
    return bri.OverlapOp(L, W, kl_n=n, rho=1.0, max_iter=3000, tbc=tbc, **kw)


@pytest.mark.parametrize("n", [1, 3, 8])
def test_upper_diagonal_apply_and_sign(n):
    need_gpu()
    U, Wo = field(L4, "cfg1")
    b = synth.gaussian_source(L4, synth.SOURCE_SEED_BASE + 21)
    op = _op(L4, U, n, kind=bri.KL_UPPER)
    out, st = op.apply(bri.spinor_to_device(b))
    ref, _, _ = oracle.ov_apply(L4, Wo, 1.0, n, b[0], tol=1e-13, kind="upper")
    assert rel_l2(bri.spinor_to_host(out)[0], ref) < TOL, st.shift_iters
    s_out, _ = op.sign(bri.spinor_to_device(b))
    sref, _, _ = oracle.sign_apply(L4, Wo, 1.0, n, b[0], tol=1e-13, kind="upper")
    assert rel_l2(bri.spinor_to_host(s_out)[0], sref) < TOL


def test_upper_diagonal_non_cubic_antiperiodic_and_mixed():
    need_gpu()
    L = (4, 4, 4, 8)
    U = synth.random_links(L, 0.4, 93)
    Wo = oracle.links(L, U, tbc=1)
    b = synth.gaussian_source(L, 94)
    ref, _, _ = oracle.ov_apply(L, Wo, 1.0, 5, b[0], tol=1e-13, kind="upper")
    op = _op(L, U, 5, tbc=1, kind=bri.KL_UPPER)
    out, _ = op.apply(bri.spinor_to_device(b))
    assert rel_l2(bri.spinor_to_host(out)[0], ref) < TOL
    Ud = bri.links_to_device(U)
    W = bri.build_links(L, Ud, bri.F64, tbc=1)
    W32 = bri.build_links(L, Ud, bri.F32, tbc=1)
    opm = bri.OverlapOp(L, W, kl_n=5, rho=1.0, tol=1e-12, max_iter=3000, tbc=1, Wlo=W32, inner=bri.F32,
                        kind=bri.KL_UPPER)
    outm, stm = opm.apply(bri.spinor_to_device(b))
    assert rel_l2(bri.spinor_to_host(outm)[0], ref) < TOL, stm.refine


@pytest.mark.parametrize("tbc", [0, 1])
def test_upper_diagonal_gradient(tbc):
    need_gpu()
    U, _ = field(L4, "cfg1", tbc)
    rng = np.random.default_rng(31 + tbc)
    chi, psi = _rand_spinor(rng, 256), _rand_spinor(rng, 256)
    n = 4
    Fref, gref = oracle.ov_force(L4, U, tbc, 1.0, n, chi, psi, tol=1e-13, kind="upper")
    Ud = bri.links_to_device(U)
    op = _op(L4, U, n, tbc=tbc, kind=bri.KL_UPPER)
    F, _, gpsi, st = op.grad(Ud, _dev(chi), _dev(psi))
    assert np.abs(_force_host(F) - Fref).max() <= 1e-9 * np.abs(Fref).max(), st.shift_iters
    assert rel_l2(bri.spinor_to_host(gpsi[None])[0], gref) < TOL


@pytest.mark.parametrize("kind", [bri.KL_DIAG, bri.KL_UPPER])
def test_relaxed_stopping_4_4(kind):
    need_gpu()
    U, Wo = field(L4, "cfg1")
    n, tol = 8, 1e-9
    kname = "diag" if kind == bri.KL_DIAG else "upper"
    c0, om, sg = oracle.kl_coeffs(n, kname)
    wmax = max(om)
    b = synth.gaussian_source(L4, synth.SOURCE_SEED_BASE + 22)
    strict = _op(L4, U, n, tol=tol, kind=kind)
    relax = _op(L4, U, n, tol=tol, kind=kind, relax=True)
    ys, sts = strict.sign(bri.spinor_to_device(b))
    yr, str_ = relax.sign(bri.spinor_to_device(b))
    for i in range(n):
        assert str_.rel_resid[i] <= tol * wmax / om[i]
        assert str_.shift_iters[i] <= sts.shift_iters[i]
    assert str_.iters <= sts.iters
    # dense exact g(H) b; the error of X r(A) b is at most |X| sum_i omega_i |r_i| / sigma_i
    d = odense.DenseOverlap(oracle.dense_matrix(L4, Wo, -1.0), 256, 1.0)
    exact = d.apply_fn(lambda lam: lam * (c0 + sum(o / (lam * lam + s) for o, s in zip(om, sg))),
                       b[0].ravel()).reshape(b[0].shape)
    xnorm = np.linalg.norm(oracle.dense_matrix(L4, Wo, -1.0), 2)
    bound = xnorm * sum(o * r / s for o, r, s in zip(om, str_.rel_resid, sg)) * np.linalg.norm(b[0])
    assert np.linalg.norm(bri.spinor_to_host(yr)[0] - exact) <= bound * 1.01 + 1e-12


def test_relaxed_stopping_bench_lattice():
    """16^4 smeared field, [16/16] at tol 1e-12: the relaxed apply stops earlier and differs
    from the strict one by less than the residual bound."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, _ = field(L, "cfg2")
    b = bri.spinor_to_device(synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 2))
    strict = _op(L, U, 16)
    relax = _op(L, U, 16, relax=True)
    ys, sts = strict.apply(b)
    yr, str_ = relax.apply(b)
    c0, om, sg = oracle.kl_coeffs(16)
    assert str_.iters <= sts.iters
    # both applies err by at most |X| sum_i omega_i |r_i| / sigma_i (rho = 1, |b| = 1); |X| <= 3 here
    bound = 3.0 * sum(o * (r1 + r2) / s for o, r1, r2, s in zip(om, str_.rel_resid, sts.rel_resid, sg))
    diff = (torch.linalg.vector_norm(yr - ys) / torch.linalg.vector_norm(b)).item()
    assert diff <= bound, (diff, bound)


def _bound_weights(om, sg):
    return [o / (2.0 * np.sqrt(s)) for o, s in zip(om, sg)]


@pytest.mark.parametrize("kind", [bri.KL_DIAG, bri.KL_UPPER])
def test_result_bound_stopping_4_4(kind):
    need_gpu()
    U, Wo = field(L4, "cfg1")
    n, tol = 8, 1e-9
    kname = "diag" if kind == bri.KL_DIAG else "upper"
    c0, om, sg = oracle.kl_coeffs(n, kname)
    w = _bound_weights(om, sg)
    b = np.concatenate([synth.gaussian_source(L4, synth.SOURCE_SEED_BASE + 23), synth.point_sources_12(L4)[[0, 7]]])
    d = odense.DenseOverlap(oracle.dense_matrix(L4, Wo, -1.0), 256, 1.0)

    def exact(r):
        return d.apply_fn(lambda lam: lam * (c0 + sum(o / (lam * lam + s) for o, s in zip(om, sg))),
                          b[r].ravel()).reshape(b[r].shape)

    refs = [exact(r) for r in range(3)]
    bd = bri.spinor_to_device(b)
    op = _op(L4, U, n, tol=tol, kind=kind, relax=bri.RELAX_BOUND)
    strict = _op(L4, U, n, tol=tol, kind=kind)
    for r in range(3):
        y, st = op.sign(bd[r:r + 1].contiguous())
        assert sum(wi * st.rel_resid[i] for i, wi in enumerate(w)) <= tol * (1 + 1e-9), st.rel_resid
        err = np.linalg.norm(bri.spinor_to_host(y)[0] - refs[r]) / np.linalg.norm(b[r])
        assert err <= tol, (r, err)
        _, sts = strict.sign(bd[r:r + 1].contiguous())
        assert st.iters <= sts.iters
    opb = _op(L4, U, n, tol=tol, kind=kind, relax=bri.RELAX_BOUND, nrhs=3)
    yb, _ = opb.sign(bd)
    yb = bri.spinor_to_host(yb)
    for r in range(3):
        assert np.linalg.norm(yb[r] - refs[r]) / np.linalg.norm(b[r]) <= tol, r
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64)
    W32 = bri.build_links(L4, Ud, bri.F32)
    opm = bri.OverlapOp(L4, W, kl_n=n, rho=1.0, tol=tol, max_iter=3000, Wlo=W32, inner=bri.F32, kind=kind,
                        relax=bri.RELAX_BOUND, nrhs=3)
    ym, stm = opm.sign(bd)
    ym = bri.spinor_to_host(ym)
    for r in range(3):
        err = np.linalg.norm(ym[r] - refs[r]) / np.linalg.norm(b[r])
        assert err <= 2 * tol, (r, err, stm.refine)


def test_result_bound_bench_lattice():
    """16^4 smeared field, [16/16]: the result bound at 1e-11 against the strict apply at 1e-13,
    in FP64 and with the FP32 low-precision phase."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, _ = field(L, "cfg2")
    b = bri.spinor_to_device(synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 2))
    tol = 1e-11
    ref, st_ref = _op(L, U, 16, tol=1e-13).apply(b)
    _, st12 = _op(L, U, 16, tol=1e-12).apply(b)
    yb, stb = _op(L, U, 16, tol=tol, relax=bri.RELAX_BOUND).apply(b)
    _, om, sg = oracle.kl_coeffs(16)
    w = _bound_weights(om, sg)
    # the strict reference errs by at most sum_i w_i 1e-13 itself (rho = 1, |b| = 1)
    slack = sum(w) * 1e-13
    diff = (torch.linalg.vector_norm(yb - ref) / torch.linalg.vector_norm(b)).item()
    print(f"bound 1e-11: {stb.iters} iterations (strict 1e-12: {st12.iters}), difference {diff:.1e}", flush=True)
    assert sum(wi * stb.rel_resid[i] for i, wi in enumerate(w)) <= tol * (1 + 1e-9)
    assert diff <= tol + slack, diff
    assert stb.iters < st12.iters
    Ud = bri.links_to_device(U)
    W = bri.build_links(L, Ud, bri.F64)
    W32 = bri.build_links(L, Ud, bri.F32)
    opm = bri.OverlapOp(L, W, kl_n=16, rho=1.0, tol=tol, max_iter=3000, Wlo=W32, inner=bri.F32,
                        relax=bri.RELAX_BOUND)
    ym, stm = opm.apply(b)
    diffm = (torch.linalg.vector_norm(ym - ref) / torch.linalg.vector_norm(b)).item()
    print(f"bound 1e-11, FP32 phase: {stm.iters} iterations ({stm.refine} in FP32), difference {diffm:.1e}",
          flush=True)
    assert diffm <= 2 * tol + slack, diffm
