"""GPU parity of the operator-quality measures of Sec. 7 (normality defect, Ginsparg-Wilson
defect, locality profile) for the f_{1,1} overlap D = D^(1)_{-1} + 1 (Kenney-Laub n = 1,
rho = 1) with the Brillouin and Wilson kernels, c_SW = 0 and 1: the library's measures against
the same expressions evaluated with the oracle's dense overlap matrix on the same vectors."""

import numpy as np
import pytest

import oracle
import paper_1701_00726_amd as bri
import synth
from oracle import dense as odense
from oracle import kl
from paper_1701_00726_amd import quality
from tests._gpu import field, need_gpu, torch

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)


def _dense_ov(K, n=1, rho=1.0):
    d = odense.DenseOverlap(oracle.dense_matrix(L4, K, -rho), 256, rho)
    G = d.fn_of_H(lambda lam: lam * kl.r_diag_f64(lam * lam, n))
    return rho * (np.eye(3072) + d.G5[:, None] * G), np.diag(d.G5)


@pytest.mark.parametrize("kernel", [bri.KERNEL_BRILLOUIN, bri.KERNEL_WILSON])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_defects_and_locality_against_dense(kernel, csw):
    need_gpu()
    U, Wo = field(L4, "cfg1")
    C = oracle.clover_field(L4, U, csw) if csw else None
    if kernel == bri.KERNEL_BRILLOUIN:
        K = oracle.BrillouinKernel(Wo, C)
    else:
        K = oracle.WilsonKernel(U, 0, C)
    D, G5 = _dense_ov(K)
    W = bri.build_links(L4, bri.links_to_device(U), bri.F64, csw=csw)
    op = bri.OverlapOp(L4, W, kl_n=1, rho=1.0, tol=1e-13, max_iter=5000, kernel=kernel, nrhs=3)
    eta_h = synth.gaussian_source(L4, synth.SOURCE_SEED_BASE + 80, nrhs=3)
    eta = bri.spinor_to_device(eta_h)
    norm_gpu = quality.normality_defect(op, eta)
    gw_gpu = quality.gw_defect(op, eta)
    Dd = D.conj().T
    for c in range(3):
        e = eta_h[c].ravel()
        norm_ref = np.linalg.norm(D @ (Dd @ e) - Dd @ (D @ e))
        gw_ref = np.linalg.norm(D @ (G5 @ e) + G5 @ (D @ e) - D @ (G5 @ (D @ e)))
        assert abs(norm_gpu[c] - norm_ref) <= 1e-9 * max(norm_ref, 1e-3), (c, norm_gpu[c], norm_ref)
        assert abs(gw_gpu[c] - gw_ref) <= 1e-9 * max(gw_ref, 1e-3), (c, gw_gpu[c], gw_ref)
        assert norm_ref > 1e-6 and gw_ref > 1e-6  # f_{1,1} is far from the exact sign
    eta0 = quality.point_source(L4, 5)
    r, mag = quality.locality_profile(op, L4, eta0)
    e0 = bri.spinor_to_host(eta0)[0].ravel()
    ref = np.linalg.norm((D @ e0).reshape(256, 12), axis=1)
    assert np.abs(mag - ref).max() <= 1e-10 * ref.max()
    assert r[0] == 0 and mag.argmax() == 0
