"""Pins of the oracle's Wilson kernel (eq. (def_wils), c_SW = 0) and of the overlap built on it:

  * free-field plane waves against the momentum form of App. A (nabla^std = i sin p,
    lap^std = 2 sum cos p - 8), periodic and antiperiodic in t, non-cubic lattices;
  * the 16 corners of the Brillouin zone: D = 2k + m0 with k momentum components at pi (the
    doublers the Laplacian term lifts);
  * gauge covariance, the adjoint identity, gamma5-hermiticity (checked, since the oracle's
    adjoint is the transposed sum), the antiperiodic sign, dense matrix against the apply;
  * the Wilson overlap: the per-shift rational against the dense eigendecomposition, and with
    the exact sign function the Ginsparg-Wilson relation and eigenvalues on the circle
    |lambda - rho| = rho.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import dense as odense
from oracle import kl
from tests._lattice import plane_wave, shift_index
from tests.test_oracle_operator import _gauge


def _wilson_symbol(p, m0):
    p = np.asarray(p, dtype=np.float64)
    D = (m0 + np.sum(1 - np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        D = D + 1j * np.sin(p[mu]) * oracle.gamma(mu)
    return D


@pytest.mark.parametrize("L,tbc", [((4, 4, 4, 4), 0), ((4, 6, 2, 8), 0), ((6, 4, 4, 6), 1)])
def test_free_field_plane_waves(L, tbc):
    K = oracle.WilsonKernel(synth.unit_links(L), tbc)
    rng = np.random.default_rng(15)
    m0 = -0.61
    for _ in range(6):
        n = np.array([rng.integers(0, L[mu]) for mu in range(4)])
        p = 2 * np.pi * n / np.asarray(L)
        if tbc:
            p[3] = (2 * n[3] + 1) * np.pi / L[3]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        got = oracle.dirac(L, K, m0, plane_wave(L, p, u))
        want = plane_wave(L, p, _wilson_symbol(p, m0) @ u)
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max(), (L, p)


def test_doublers():
    L = (4, 4, 4, 4)
    K = oracle.WilsonKernel(synth.unit_links(L))
    u = np.arange(12, dtype=np.complex128).reshape(4, 3) + 1
    for corner in itertools.product([0, 1], repeat=4):
        p = np.pi * np.asarray(corner)
        got = oracle.dirac(L, K, 0.0, plane_wave(L, p, u))
        want = 2.0 * sum(corner) * plane_wave(L, p, u)
        assert np.abs(got - want).max() < 1e-14 * max(1.0, np.abs(want).max())


@pytest.fixture(scope="module")
def rough():
    L = (4, 4, 6, 4)
    U = synth.random_links(L, 0.8, 12)
    return L, U


@pytest.mark.parametrize("tbc", [0, 1])
def test_adjoint_gamma5_hermiticity_and_dense(rough, tbc):
    L, U = rough
    K = oracle.WilsonKernel(U, tbc)
    m0 = -1.0
    psi = synth.gaussian_source(L, 14)[0]
    phi = synth.gaussian_source(L, 15)[0]
    Dpsi = oracle.dirac(L, K, m0, psi)
    Dadj_phi = oracle.dirac_adj(L, K, m0, phi)
    assert abs(np.vdot(phi, Dpsi) - np.vdot(Dadj_phi, psi)) < 1e-13
    g5Dg5 = oracle.gamma5_apply(oracle.dirac(L, K, m0, oracle.gamma5_apply(phi)))
    assert np.abs(g5Dg5 - Dadj_phi).max() < 1e-14
    M = oracle.dense_matrix(L, K, m0)
    assert np.abs(M @ psi.ravel() - Dpsi.ravel()).max() < 1e-13
    # 9-point stencil: 1 diagonal block and 8 neighbour blocks per row block of 12
    assert np.count_nonzero(np.abs(M[:12]).sum(axis=0) > 0) <= 9 * 12


def test_gauge_covariance_and_antiperiodic_sign(rough):
    L, U = rough
    V = int(np.prod(L))
    G = synth.random_su3(V, 2.0, 98)
    psi = synth.gaussian_source(L, 16)[0]
    m0 = -1.0
    lhs = oracle.dirac(L, oracle.WilsonKernel(_gauge(L, U, G)), m0, np.einsum("xab,xsb->xsa", G, psi))
    rhs = np.einsum("xab,xsb->xsa", G, oracle.dirac(L, oracle.WilsonKernel(U), m0, psi))
    assert np.abs(lhs - rhs).max() < 1e-13
    # antiperiodic in t = periodic with the t links of the last slice negated
    Uf = U.copy()
    per_t = V // L[3]
    Uf[3, V - per_t:] *= -1
    a = oracle.dirac(L, oracle.WilsonKernel(U, 1), m0, psi)
    b = oracle.dirac(L, oracle.WilsonKernel(Uf, 0), m0, psi)
    assert np.abs(a - b).max() < 1e-14


def test_wilson_overlap_rational_and_exact_sign():
    L = (4, 4, 4, 4)
    U = synth.random_links(L, 0.3, synth.LINK_SEED_BASE + 1)
    K = oracle.WilsonKernel(U)
    rho, n = 1.0, 8
    d = odense.DenseOverlap(oracle.dense_matrix(L, K, -rho), 256, rho)
    b = synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 5)[0]
    got, _, rel = oracle.ov_apply(L, K, rho, n, b, tol=1e-13)
    want = b.ravel() + d.G5 * d.apply_fn(lambda lam: lam * kl.r_diag_f64(lam * lam, n), b.ravel())
    assert np.linalg.norm(got.ravel() - rho * want) <= 1e-11 * np.linalg.norm(want)
    # exact sign: Ginsparg-Wilson and the eigenvalues on the circle |lambda - rho| = rho
    S = d.fn_of_H(np.sign)
    Dov = rho * (np.eye(3072) + d.G5[:, None] * S)
    G5 = np.diag(d.G5)
    gw = Dov @ G5 + G5 @ Dov - Dov @ G5 @ Dov / rho
    assert np.abs(gw).max() < 1e-11
    ev = np.linalg.eigvals(Dov)
    assert np.abs(np.abs(ev - rho) - rho).max() < 1e-10
