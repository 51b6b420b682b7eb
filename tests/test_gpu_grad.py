"""GPU parity of the differentiation path (Sec. 9 force, App. C.1 links).

  * bri_link_grad against the oracle's path-by-path product rule on 4^4
    (periodic and antiperiodic, several weighted pairs), element by element;
  * the complex link gradient GU against directional derivatives of the
    oracle's forward operator, and against the force (F = Re tr(conj(GU)^T X U));
  * the same at 16^4 with point-supported pairs, so the oracle visits one site;
  * ov_apply_grad against the oracle's partial-fraction gradient on 4^4, and
    grad_psi against D_ov^dag chi = gamma5 D_ov gamma5 chi from the oracle;
  * the torch.autograd.Function wrappers against the kernels and against
    directional differences of their own forward passes.

Tolerances: the force is a sum of O(10^4) FP64 terms per link; 1e-12 of
max |F| for the Brillouin force, 1e-9 for the overlap force, whose shift
solutions carry the CG tolerance 1e-12 (1e-13 on the oracle side).
"""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import field, need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)


def _rand_spinor(rng, V):
    return rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))


def _dev(psi):
    """(V, 4, 3) numpy -> (4, 3, V) device tensor."""
    return bri.spinor_to_device(psi[None])[0]


def _force_host(F_t):
    """(4, 8, V) tensor -> (4, V, 8) numpy, the oracle's layout."""
    return np.ascontiguousarray(np.transpose(F_t.cpu().numpy(), (0, 2, 1)))


def _gu_host(GU_t):
    """(4, 3, 3, V) tensor -> (4, V, 3, 3) numpy."""
    return np.ascontiguousarray(np.transpose(GU_t.cpu().numpy(), (0, 3, 1, 2)))


def _force_from_gu(U, GU):
    """F^a = Re sum_ab conj(GU)_ab (i lambda_a U / 2)_ab."""
    F = np.zeros(U.shape[:2] + (8,))
    for a in range(8):
        lam = oracle.gell_mann(a)
        dU = np.einsum("ij,mxjk->mxik", 0.5j * lam, U)
        F[..., a] = np.einsum("mxij,mxij->mx", np.conj(GU), dU).real
    return F


@pytest.mark.parametrize("tbc", [0, 1])
@pytest.mark.parametrize("kind", ["rough", "cfg2"])
def test_link_force_4_4(kind, tbc):
    need_gpu()
    U, _ = field(L4, kind, tbc)
    V = 256
    rng = np.random.default_rng(40 + tbc)
    pairs = [(w, _rand_spinor(rng, V), _rand_spinor(rng, V)) for w in (1.0, -0.37, 2.5)]
    ref = oracle.link_force(L4, U, tbc, pairs)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64, tbc=tbc)
    F, GU = bri.link_grad(L4, Ud, W, [(w, _dev(u), _dev(v)) for w, u, v in pairs], tbc=tbc, force=True,
                          link_grad=True)
    got = _force_host(F)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # the link gradient carries the same information
    gu = _gu_host(GU)
    assert np.abs(_force_from_gu(U, gu) - ref).max() <= 1e-12 * np.abs(ref).max()
    # directional derivative of the oracle's forward operator along a random non-unitary dU
    dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)

    def S(Ux):
        Wx = oracle.links(L4, Ux, tbc)
        return sum(w * np.vdot(u, oracle.dirac(L4, Wx, -0.4, v)).real for w, u, v in pairs)

    h = 1e-4
    fd = (-S(U + 2 * h * dU) + 8 * S(U + h * dU) - 8 * S(U - h * dU) + S(U - 2 * h * dU)) / (12 * h)
    lin = np.sum(np.conj(gu) * dU).real
    assert abs(fd - lin) <= 1e-8 * abs(lin)


def test_link_force_16_4_point_pairs():
    need_gpu()
    L = (16, 16, 16, 16)
    V = 16**4
    U = synth.random_links(L, 0.5, synth.LINK_SEED_BASE + 3)
    rng = np.random.default_rng(5)
    pairs = []
    for k, x0 in enumerate((0, V - 1, 12345)):
        u = np.zeros((V, 4, 3), complex)
        u[x0] = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        pairs.append((1.0 + k, u, _rand_spinor(rng, V)))
    ref = oracle.link_force(L, U, 1, pairs)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L, Ud, bri.F64, tbc=1)
    F, _ = bri.link_grad(L, Ud, W, [(w, _dev(u), _dev(v)) for w, u, v in pairs], tbc=1)
    got = _force_host(F)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.count_nonzero(np.abs(ref) > 0) > 1000  # the three sites reach many links


@pytest.mark.parametrize("tbc", [0, 1])
def test_overlap_grad_4_4(tbc):
    need_gpu()
    U, Wo = field(L4, "cfg1", tbc)
    rng = np.random.default_rng(7 + tbc)
    chi, psi = _rand_spinor(rng, 256), _rand_spinor(rng, 256)
    n, rho = 6, 1.0
    Fref, gref = oracle.ov_force(L4, U, tbc, rho, n, chi, psi, tol=1e-13)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64, tbc=tbc)
    op = bri.OverlapOp(L4, W, kl_n=n, rho=rho, tol=1e-12, tbc=tbc)
    F, GU, gpsi, st = op.grad(Ud, _dev(chi), _dev(psi), force=True, link_grad=True)
    got = _force_host(F)
    assert np.abs(got - Fref).max() <= 1e-9 * np.abs(Fref).max(), st.shift_iters
    assert np.abs(_force_from_gu(U, _gu_host(GU)) - Fref).max() <= 1e-9 * np.abs(Fref).max()
    g = bri.spinor_to_host(gpsi[None])[0]
    assert rel_l2(g, gref) < 1e-10
    # D_ov^dag chi = gamma5 D_ov gamma5 chi (gamma5-hermiticity of D_ov, Sec. 4)
    g5chi = oracle.gamma5_apply(chi)
    dg, _, _ = oracle.ov_apply(L4, Wo, rho, n, g5chi, tol=1e-13)
    assert rel_l2(g, oracle.gamma5_apply(dg)) < 1e-10
    assert st.iters > 0 and max(st.rel_resid) <= 1e-12


def test_brillouin_autograd():
    need_gpu()
    U, _ = field(L4, "cfg2", 1)
    rng = np.random.default_rng(9)
    Ud = bri.links_to_device(U).requires_grad_(True)
    psi = bri.spinor_to_device(np.stack([_rand_spinor(rng, 256) for _ in range(2)])).requires_grad_(True)
    chi = bri.spinor_to_device(np.stack([_rand_spinor(rng, 256) for _ in range(2)]))
    out = bri.BrillouinApply.apply(Ud, psi, L4, -0.5, 1)
    loss = torch.sum(torch.conj(chi) * out).real
    loss.backward()
    with torch.no_grad():
        W = bri.build_links(L4, Ud.detach(), bri.F64, tbc=1)
        want_psi = bri.apply_dag(L4, W, bri.F64, -0.5, chi)
        _, want_U = bri.link_grad(L4, Ud.detach(), W, [(1.0, chi[r], psi[r].detach()) for r in range(2)], tbc=1,
                                  force=False, link_grad=True)
    assert torch.allclose(psi.grad, want_psi, rtol=0, atol=1e-12 * want_psi.abs().max().item())
    assert torch.allclose(Ud.grad, want_U, rtol=0, atol=1e-12 * want_U.abs().max().item())
    # directional difference of the forward pass itself
    dU = torch.randn_like(Ud.detach())
    dpsi = torch.randn_like(psi.detach())
    h = 1e-4

    def L_at(t):
        with torch.no_grad():
            o = bri.BrillouinApply.apply(Ud.detach() + t * dU, psi.detach() + t * dpsi, L4, -0.5, 1)
            return torch.sum(torch.conj(chi) * o).real.item()

    fd = (-L_at(2 * h) + 8 * L_at(h) - 8 * L_at(-h) + L_at(-2 * h)) / (12 * h)
    lin = (torch.sum(torch.conj(Ud.grad) * dU).real + torch.sum(torch.conj(psi.grad) * dpsi).real).item()
    assert abs(fd - lin) <= 1e-8 * abs(lin)


def test_overlap_autograd():
    need_gpu()
    U, _ = field(L4, "cfg1", 0)
    rng = np.random.default_rng(13)
    Ud = bri.links_to_device(U).requires_grad_(True)
    psi = _dev(_rand_spinor(rng, 256)).requires_grad_(True)
    chi = _dev(_rand_spinor(rng, 256))
    kw = dict(kl_n=6, rho=1.0, tol=1e-13, max_iter=4000, tbc=0)
    out = bri.OverlapApply.apply(Ud, psi, L4, **kw)
    loss = torch.sum(torch.conj(chi) * out).real
    loss.backward()
    dU = torch.randn_like(Ud.detach())
    dpsi = torch.randn_like(psi.detach())
    h = 1e-4

    def L_at(t):
        with torch.no_grad():
            o = bri.OverlapApply.apply(Ud.detach() + t * dU, psi.detach() + t * dpsi, L4, **kw)
            return torch.sum(torch.conj(chi) * o).real.item()

    fd = (-L_at(2 * h) + 8 * L_at(h) - 8 * L_at(-h) + L_at(-2 * h)) / (12 * h)
    lin = (torch.sum(torch.conj(Ud.grad) * dU).real + torch.sum(torch.conj(psi.grad) * dpsi).real).item()
    assert abs(fd - lin) <= 1e-7 * abs(lin)


@pytest.mark.parametrize("inner", [bri.F32, bri.F32_BF16W])
def test_overlap_grad_low_precision_inner(inner):
    """Shift solves whose late iterations run in low precision give the FP64 gradient to the
    solver tolerance."""
    need_gpu()
    U, _ = field(L4, "cfg1", 1)
    rng = np.random.default_rng(17)
    chi, psi = _dev(_rand_spinor(rng, 256)), _dev(_rand_spinor(rng, 256))
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64, tbc=1)
    F64_, _, g64, _ = bri.OverlapOp(L4, W, kl_n=6, tol=1e-12, tbc=1).grad(Ud, chi, psi)
    lo = bri.build_links(L4, Ud, inner, tbc=1)
    op = bri.OverlapOp(L4, W, kl_n=6, tol=1e-12, tbc=1, Wlo=lo, inner=inner)
    F, _, g, st = op.grad(Ud, chi, psi)
    assert float((F - F64_).abs().max()) <= 1e-9 * float(F64_.abs().max())
    assert float(torch.linalg.vector_norm(g - g64) / torch.linalg.vector_norm(g64)) < 1e-10
    assert st.refine >= (1 if inner == bri.F32 else 0) and max(st.rel_resid) <= 1e-12


def test_grad_error_paths():
    need_gpu()
    U, _ = field(L4, "cfg1", 0)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64)
    z = torch.zeros((4, 3, 256), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        bri.link_grad(L4, Ud, W, [])
    with pytest.raises(ValueError):
        bri.link_grad(L4, Ud, W, [(1.0, z, z)], force=False, link_grad=False)
    # a zero source gives zero gradients
    op = bri.OverlapOp(L4, W, kl_n=4)
    F, _, g, _ = op.grad(Ud, z, z)
    assert float(F.abs().max()) == 0.0 and float(g.abs().max()) == 0.0


def test_overlap_grad_directional_at_bench_size():
    """16^4 smeared field, [16/16]: the link gradient and D_ov^dag chi against five-point
    directional differences of the library's own forward apply (CG tolerance 1e-13), along a
    random complex direction in the links and in psi."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, _ = field(L, "cfg2", 1)
    Ud = bri.links_to_device(U)
    V = 16**4
    rng = np.random.default_rng(21)
    chi = bri.spinor_to_device(synth.gaussian_source(L, 5))[0]
    psi = bri.spinor_to_device(synth.gaussian_source(L, 6))[0]
    kw = dict(kl_n=16, rho=1.0, tol=1e-13, max_iter=4000, tbc=1)
    W = bri.build_links(L, Ud, bri.F64, tbc=1)
    op = bri.OverlapOp(L, W, **{k: v for k, v in kw.items()})
    F, GU, gpsi, st = op.grad(Ud, chi, psi, force=True, link_grad=True)
    assert max(st.rel_resid) <= 1e-13
    dU = torch.randn_like(Ud) * 1e-2
    dpsi = torch.randn_like(psi)
    h = 1e-3

    def S(t):
        Ut = Ud + t * dU
        Wt = bri.build_links(L, Ut, bri.F64, tbc=1)
        o, _ = bri.OverlapOp(L, Wt, **kw).apply((psi + t * dpsi).reshape(1, 4, 3, V).contiguous())
        return torch.sum(torch.conj(chi) * o[0]).real.item()

    fd = (-S(2 * h) + 8 * S(h) - 8 * S(-h) + S(-2 * h)) / (12 * h)
    lin = (torch.sum(torch.conj(GU) * dU).real + torch.sum(torch.conj(gpsi) * dpsi).real).item()
    assert abs(fd - lin) <= 1e-7 * abs(lin), (fd, lin)
    # the force is the projection of the same gradient onto i lambda_a U / 2
    Fh = _force_host(F)
    assert np.abs(_force_from_gu(U, _gu_host(GU)) - Fh).max() <= 1e-12 * np.abs(Fh).max()


@pytest.mark.parametrize("tbc", [0, 1])
def test_overlap_grad_recompute_4_4(tbc):
    """Shift solutions recomputed (the shifts solved 1 and 4 at a time, keeping only those) give
    the force and D_ov^dag chi of the stored mode and of the oracle (Sec. 9 force of the
    partial fractions)."""
    need_gpu()
    U, _ = field(L4, "cfg1", tbc)
    rng = np.random.default_rng(31 + tbc)
    chi, psi = _rand_spinor(rng, 256), _rand_spinor(rng, 256)
    n, rho = 6, 1.0
    Fref, gref = oracle.ov_force(L4, U, tbc, rho, n, chi, psi, tol=1e-13)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L4, Ud, bri.F64, tbc=tbc)
    Fs, _, gs, _ = bri.OverlapOp(L4, W, kl_n=n, rho=rho, tol=1e-12, tbc=tbc).grad(Ud, _dev(chi), _dev(psi))
    for m in (1, 4):
        op = bri.OverlapOp(L4, W, kl_n=n, rho=rho, tol=1e-12, tbc=tbc, recompute=m)
        F, _, g, st = op.grad(Ud, _dev(chi), _dev(psi))
        got = _force_host(F)
        assert np.abs(got - Fref).max() <= 1e-9 * np.abs(Fref).max(), m
        assert np.abs(got - _force_host(Fs)).max() <= 1e-9 * np.abs(Fref).max(), m
        gh = bri.spinor_to_host(g[None])[0]
        assert rel_l2(gh, gref) < 1e-10 and rel_l2(gh, bri.spinor_to_host(gs[None])[0]) < 1e-10
        assert max(st.rel_resid) <= 1e-12 and all(i > 0 for i in st.shift_iters)
        # every shift solved in its own group (m = 1) takes more iterations than one multi-shift
        if m == 1:
            assert st.iters > max(st.shift_iters)


def test_overlap_grad_recompute_16_4():
    """The gradient workload (16^4, [16/16]) with the shift solutions recomputed four at a time:
    force and D_ov^dag chi against the stored mode, and a smaller workspace."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, _ = field(L, "cfg2", 0)
    Ud = bri.links_to_device(U)
    chi = bri.spinor_to_device(synth.gaussian_source(L, 7))[0]
    psi = bri.spinor_to_device(synth.gaussian_source(L, 8))[0]
    W = bri.build_links(L, Ud, bri.F64)
    ops = {m: bri.OverlapOp(L, W, kl_n=16, rho=1.0, tol=1e-12, recompute=m) for m in (0, 4)}
    out = {m: op.grad(Ud, chi, psi) for m, op in ops.items()}
    F0, _, g0, _ = out[0]
    F4, _, g4, st4 = out[4]
    assert float((F4 - F0).abs().max()) <= 1e-9 * float(F0.abs().max())
    assert float(torch.linalg.vector_norm(g4 - g0) / torch.linalg.vector_norm(g0)) < 1e-10
    assert max(st4.rel_resid) <= 1e-12
    assert ops[4]._gwork.numel() < ops[0]._gwork.numel()
