"""Pins of the oracle's clover term -(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu (eqs. (def_wils),
(def_bril)) with the clover-leaf F_mu_nu, sigma_mu_nu = (i/2)[gamma_mu, gamma_nu]:

  * unit links: F = 0, so the term vanishes;
  * a constant abelian field in one plane (flux quantised for the periodic torus): every
    plaquette is exp(+i B lambda), so F_01 = sin(B lambda) exactly and the term is
    -(c_SW/2) sigma_01 (x) sin(B lambda) at every site, which fixes orientation and sign;
  * per site the 12 x 12 block is hermitian, commutes with gamma5 (so the operator stays
    gamma5-hermitian) and is traceless in colour; it is gauge covariant;
  * with the term, D^dag (transposed sum) = gamma5 D gamma5 for both kernels, and the
    per-shift rational of the clover-improved overlap matches the dense eigendecomposition.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import dense as odense
from oracle import kl
from tests.test_oracle_operator import _gauge

CSW = 1.0


def test_unit_links_give_no_clover_term():
    L = (4, 4, 4, 4)
    C = oracle.clover_field(L, synth.unit_links(L), CSW)
    assert np.abs(C).max() == 0.0


def _abelian_field(L, k, lam):
    """U_0(x) = exp(-i B x_1 lam), U_1(x) = exp(+i B L_1 x_0 lam) on the last x_1 slice (else 1),
    B = 2 pi k / (L_0 L_1): every 0-1 plaquette U_0(x) U_1(x+0) U_0(x+1)^dag U_1(x)^dag equals
    exp(+i B lam)."""
    V = int(np.prod(L))
    B = 2 * np.pi * k / (L[0] * L[1])
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    s = np.arange(V)
    x0, x1 = s % L[0], (s // L[0]) % L[1]
    U[0] = np.array([np.diag(np.exp(-1j * B * x * lam)) for x in x1])
    edge = x1 == L[1] - 1
    U[1][edge] = np.array([np.diag(np.exp(1j * B * L[1] * x * lam)) for x in x0[edge]])
    return U, B


def test_constant_abelian_field_closed_form():
    L = (4, 6, 2, 2)
    lam = np.array([1.0, -1.0, 0.0])
    U, B = _abelian_field(L, 1, lam)
    C = oracle.clover_field(L, U, CSW)
    g = [oracle.gamma(mu) for mu in range(4)]
    sig01 = 0.5j * (g[0] @ g[1] - g[1] @ g[0])
    V = int(np.prod(L))
    s = np.arange(V)
    x0, x1 = s % L[0], (s // L[0]) % L[1]
    P = np.einsum("xab,xbc,xdc,xed->xae", U[0], U[1][(x0 + 1) % L[0] + L[0] * (s // L[0])],
                  np.conj(U[0][x0 + L[0] * ((x1 + 1) % L[1]) + L[0] * L[1] * (s // (L[0] * L[1]))]), np.conj(U[1]))
    assert np.abs(P - np.diag(np.exp(1j * B * lam))[None]).max() < 1e-14
    want = -(CSW / 2) * np.kron(sig01, np.diag(np.sin(B * lam)))
    assert np.abs(C - want[None]).max() < 1e-14
    assert np.abs(want).max() > 0.1


@pytest.fixture(scope="module")
def rough():
    L = (4, 4, 4, 6)
    U = synth.random_links(L, 0.6, 21)
    return L, U, oracle.clover_field(L, U, CSW)


def test_site_blocks_hermitian_chiral_traceless(rough):
    L, U, C = rough
    assert np.abs(C - np.conj(np.swapaxes(C, 1, 2))).max() < 1e-15
    g5 = np.kron(oracle.gamma(4), np.eye(3))
    assert np.abs(g5 @ C - C @ g5).max() < 1e-15
    # colour trace of each spin block vanishes (F traceless)
    Cs = C.reshape(-1, 4, 3, 4, 3)
    assert np.abs(np.einsum("xsata->xst", Cs)).max() < 1e-14
    assert np.abs(C).max() > 1e-2


def test_gauge_covariance(rough):
    L, U, C = rough
    V = int(np.prod(L))
    G = synth.random_su3(V, 2.0, 97)
    Cg = oracle.clover_field(L, _gauge(L, U, G), CSW)
    Gb = np.einsum("st,xab->xsatb", np.eye(4), G).reshape(V, 12, 12)
    want = Gb @ C @ np.conj(np.swapaxes(Gb, 1, 2))
    assert np.abs(Cg - want).max() < 1e-14


@pytest.mark.parametrize("kernel", ["bri", "wil"])
def test_gamma5_hermiticity_with_clover(rough, kernel):
    L, U, C = rough
    K = oracle.BrillouinKernel(oracle.links(L, U, 1), C) if kernel == "bri" else oracle.WilsonKernel(U, 1, C)
    m0 = -1.0
    psi = synth.gaussian_source(L, 31)[0]
    phi = synth.gaussian_source(L, 32)[0]
    Dpsi = oracle.dirac(L, K, m0, psi)
    Dadj = oracle.dirac_adj(L, K, m0, phi)
    assert abs(np.vdot(phi, Dpsi) - np.vdot(Dadj, psi)) < 1e-12
    assert np.abs(oracle.gamma5_apply(oracle.dirac(L, K, m0, oracle.gamma5_apply(phi))) - Dadj).max() < 1e-13
    # the term is really there
    K0 = oracle.links(L, U, 1) if kernel == "bri" else oracle.WilsonKernel(U, 1)
    assert np.abs(oracle.dirac(L, K0, m0, psi) - Dpsi).max() > 1e-2
    M = oracle.dense_matrix(L, K, m0)
    assert np.abs(M @ psi.ravel() - Dpsi.ravel()).max() < 1e-12


def test_clover_overlap_rational_against_dense():
    L = (4, 4, 4, 4)
    U = synth.random_links(L, 0.3, synth.LINK_SEED_BASE + 1)
    K = oracle.BrillouinKernel(oracle.links(L, U), oracle.clover_field(L, U, CSW))
    d = odense.DenseOverlap(oracle.dense_matrix(L, K, -1.0), 256, 1.0)
    b = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 6)[0]
    got, _, _ = oracle.ov_apply(L, K, 1.0, 6, b, tol=1e-13)
    want = b.ravel() + d.G5 * d.apply_fn(lambda lam: lam * kl.r_diag_f64(lam * lam, 6), b.ravel())
    assert np.linalg.norm(got.ravel() - want) <= 1e-11 * np.linalg.norm(want)
