"""GPU parity of bri_build_links / bri_apply / bri_apply_dag against the oracle
(App. C.1 stencil, eq. (def_bril)), through the C ABI.

Tolerances: FP64 results agree with the FP64 oracle to 1e-14 relative (L2)
and 1e-13 of the largest entry; FP32 / BF16-link results are compared with the
oracle run on the same rounded links and inputs, to 2e-6 relative (FP32
accumulation over 81 terms); the rounded links themselves must be bit-exact.
"""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from tests._gpu import field, need_gpu, rel_l2, round_links, torch

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), "rough", 0),
    ((4, 8, 4, 6), "rough", 0),
    ((4, 4, 4, 8), "rough", 1),
    ((8, 8, 8, 8), "cfg2", 0),
    # degenerate extents: +1 and -1 neighbours coincide (2), or are the site itself (1), so the
    # stored and the daggered links of several displacements meet on the same sites
    ((2, 2, 2, 8), "rough", 1),
    ((16, 4, 1, 1), "rough", 1),
    ((4, 4, 2, 2), "rough", 0),
]


@pytest.mark.parametrize("L,kind,tbc", CASES)
def test_build_links_f64(L, kind, tbc):
    need_gpu()
    U, Wo = field(L, kind, tbc)
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=tbc)
    torch.cuda.synchronize()
    Wg = bri.links_W_to_host(W)
    ref = Wo[:, :40]
    assert np.abs(Wg - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [bri.F32, bri.F32_BF16W])
def test_build_links_low_precision_bit_exact(prec):
    need_gpu()
    L = (4, 8, 4, 6)
    U, Wo = field(L, "rough")
    W = bri.build_links(L, bri.links_to_device(U), prec)
    torch.cuda.synchronize()
    Wg = bri.links_W_to_host(W, prec)
    W64 = bri.links_W_to_host(bri.build_links(L, bri.links_to_device(U), bri.F64))
    # rounding decisions are taken from the library's own FP64 links, so they must match exactly
    assert np.array_equal(Wg, round_links(W64, prec))
    assert np.abs(Wg - Wo[:, :40]).max() <= (4e-3 if prec == bri.F32_BF16W else 1e-7)


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("prec", [bri.F32, bri.F32_BF16W])
def test_round_links_equals_low_precision_build(prec, csw):
    """bri_round_links on the FP64 array gives bri_build_links' low-precision array bit for bit
    (the clover slabs too for csw != 0)."""
    need_gpu()
    L = (4, 8, 4, 6)
    U, _ = field(L, "rough")
    Ud = bri.links_to_device(U)
    W64 = bri.build_links(L, Ud, bri.F64, csw=csw)
    Wb = bri.build_links(L, Ud, prec, csw=csw)
    Wr = bri.round_links(L, W64, prec)
    torch.cuda.synchronize()
    assert Wr.shape == Wb.shape == (48 if csw else 40, 3, 3, int(np.prod(L)))
    assert np.array_equal(Wr.cpu().numpy().view(np.uint32), Wb.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("L,kind,tbc", CASES)
@pytest.mark.parametrize("dag", [False, True])
def test_apply_f64(L, kind, tbc, dag):
    need_gpu()
    U, Wo = field(L, kind, tbc)
    W = bri.build_links(L, bri.links_to_device(U), bri.F64, tbc=tbc)
    psi = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 50, nrhs=3)
    m0 = -1.0
    fn = bri.apply_dag if dag else bri.apply
    out = bri.spinor_to_host(fn(L, W, bri.F64, m0, bri.spinor_to_device(psi)))
    ref = (oracle.dirac_adj if dag else oracle.dirac)(L, Wo, m0, psi)
    assert rel_l2(out, ref) < 1e-14
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [bri.F32, bri.F32_BF16W])
@pytest.mark.parametrize("dag", [False, True])
def test_apply_low_precision(prec, dag):
    need_gpu()
    L = (8, 8, 8, 8)
    U, Wo = field(L, "cfg2")
    W64 = bri.build_links(L, bri.links_to_device(U), bri.F64)
    W = bri.build_links(L, bri.links_to_device(U), prec)
    psi = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 51, nrhs=2)
    psi32 = psi.astype(np.complex64).astype(np.complex128)
    m0 = -1.0
    fn = bri.apply_dag if dag else bri.apply
    out = bri.spinor_to_host(fn(L, W, prec, m0, bri.spinor_to_device(psi32, prec)))
    Wr = np.zeros_like(Wo)
    Wr[:, :40] = round_links(bri.links_W_to_host(W64), prec)
    # the remaining 41 displacements follow from the stored 40 (W_{80-j}(x) = W_j(x + d)^dag) and d = 0
    from tests._lattice import disp, shift_index

    Wr[:, 40] = np.eye(3)
    for j in range(40):
        Wr[shift_index(L, disp(j)), 80 - j] = np.conj(np.swapaxes(Wr[:, j], -1, -2))
    ref = (oracle.dirac_adj if dag else oracle.dirac)(L, Wr, m0, psi32)
    assert rel_l2(out, ref) < 2e-6
    # and against the unrounded FP64 operator, at the size the link rounding implies
    ref64 = (oracle.dirac_adj if dag else oracle.dirac)(L, Wo, m0, psi)
    assert rel_l2(out, ref64) < (1e-2 if prec == bri.F32_BF16W else 1e-6)


def test_free_field_doublers_on_gpu():
    """U = 1: the 15 corners p in {0, pi}^4 \\ {0} are eigenvectors with eigenvalue 2 + m0 (Sec. 5)."""
    need_gpu()
    import itertools

    from tests._lattice import plane_wave

    L = (4, 4, 4, 4)
    U, _ = field(L, "unit")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    u = (np.arange(12).reshape(4, 3) + 1.0).astype(np.complex128)
    m0 = -0.4
    for corner in itertools.product([0, 1], repeat=4):
        psi = plane_wave(L, np.pi * np.asarray(corner), u)[None]
        out = bri.spinor_to_host(bri.apply(L, W, bri.F64, m0, bri.spinor_to_device(psi)))
        lam = m0 if sum(corner) == 0 else 2 + m0
        assert np.abs(out - lam * psi).max() < 1e-13


def test_bench_size_16_4():
    """The benchmark's 16^4 smeared field, FP64 and FP32, every site."""
    need_gpu()
    L = (16, 16, 16, 16)
    U, Wo = field(L, "cfg2")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    Wg = bri.links_W_to_host(W)
    assert np.abs(Wg - Wo[:, :40]).max() <= 1e-14
    psi = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 2)
    out = bri.spinor_to_host(bri.apply(L, W, bri.F64, -1.0, bri.spinor_to_device(psi)))
    ref = oracle.dirac(L, Wo, -1.0, psi)
    assert rel_l2(out, ref) < 1e-14
    W32 = bri.build_links(L, bri.links_to_device(U), bri.F32)
    out32 = bri.spinor_to_host(bri.apply(L, W32, bri.F32, -1.0, bri.spinor_to_device(psi, bri.F32)))
    assert rel_l2(out32, ref) < 1e-6


def test_repeatable_bitwise():
    need_gpu()
    L = (8, 8, 8, 8)
    U, _ = field(L, "cfg2")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    psi = bri.spinor_to_device(synth.gaussian_source(L, 9))
    a = bri.apply(L, W, bri.F64, -1.0, psi)
    b = bri.apply(L, W, bri.F64, -1.0, psi)
    assert torch.equal(a, b)
