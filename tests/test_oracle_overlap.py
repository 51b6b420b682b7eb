"""Pins of the oracle's sign function and overlap operator.

  * 4^4 random SU(3) field: the per-shift CG evaluation of
    rho (1 + gamma5 g_{2n+1}(H)) against the dense eigendecomposition of H
    (same rational function, no Krylov solver), eq. (def_over), (KLnn_parfrac);
  * the same against the exact sign function within max |g(lam) - sgn(lam)|;
  * sign^2 = 1 within that bound; the Ginsparg-Wilson identity
    D g5 + g5 D - D g5 D / rho = rho g5 (1 - S^2) for D = rho (1 + g5 S),
    eq. (ginswils_one); normality;
  * free field: plane waves against rho [1 + X(p) r_n(pt^2 + M^2)] (App. A).
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import dense as odense
from oracle import kl
from tests._lattice import plane_wave

L4 = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def field():
    U = synth.random_links(L4, 0.3, 1701 + 1)
    W = oracle.links(L4, U)
    D = oracle.dense_matrix(L4, W, -1.0)
    return W, odense.DenseOverlap(D, 256, 1.0)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [8, 16])
def test_cg_overlap_matches_dense_rational(field, n):
    W, dov = field
    b = synth.point_source(L4)[0]
    got, iters, rel = oracle.ov_apply(L4, W, 1.0, n, b, tol=1e-13)
    assert rel.max() <= 1e-13
    want = dov.ov_apply(n, b.reshape(-1)).reshape(b.shape)
    assert _rel(got, want) < 1e-12
    g = synth.gaussian_source(L4, 726 + 1)[0]
    got_s, _, _ = oracle.sign_apply(L4, W, 1.0, n, g, tol=1e-13)
    want_s = dov.g_apply(n, g.reshape(-1)).reshape(g.shape)
    assert _rel(got_s, want_s) < 1e-12


def test_rational_against_exact_sign(field):
    W, dov = field
    lam = np.abs(dov.lam)
    assert 0.5 < lam.min() and lam.max() < 1.4  # |H| spectrum of this field
    g = synth.gaussian_source(L4, 800)[0].reshape(-1)
    exact = dov.sign_exact_apply(g)
    for n in (4, 8, 16):
        bound = dov.sign_bound(n)
        approx = dov.g_apply(n, g)
        assert np.linalg.norm(approx - exact) <= bound * np.linalg.norm(g) * (1 + 1e-6) + 1e-15
    assert dov.sign_bound(8) < 2e-10 and dov.sign_bound(16) < 1e-15


def test_sign_squared_and_ginsparg_wilson(field):
    W, dov = field
    n, rho = 8, 1.0
    eta = synth.gaussian_source(L4, 801)[0]
    S_eta, _, _ = oracle.sign_apply(L4, W, rho, n, eta, tol=1e-14)
    SS_eta, _, _ = oracle.sign_apply(L4, W, rho, n, S_eta, tol=1e-14)
    bound = dov.sign_bound(n)
    # |(1 - S^2) eta| <= max|1 - g(lam)^2| |eta| ~ 2 bound
    assert np.linalg.norm(eta - SS_eta) <= 2.5 * bound
    g5 = oracle.gamma5_apply
    Dov = lambda v: oracle.ov_apply(L4, W, rho, n, v, tol=1e-14)[0]  # noqa: E731
    lhs = Dov(g5(eta)) + g5(Dov(eta)) - Dov(g5(Dov(eta))) / rho
    rhs = rho * g5(eta - SS_eta)
    assert np.linalg.norm(lhs - rhs) < 1e-12
    # normality: D^dag = rho (1 + S g5) and [D, D^dag] = rho^2 (g5 S^2 g5 - S^2), of the size of the sign defect
    Dadj = lambda v: rho * (v + oracle.sign_apply(L4, W, rho, n, g5(v), tol=1e-14)[0])  # noqa: E731
    comm = Dov(Dadj(eta)) - Dadj(Dov(eta))
    assert np.linalg.norm(comm) <= 5 * bound + 1e-12


def _free_symbol(p, m0):
    c, s = np.cos(p), np.sin(p)
    pt = np.array([s[mu] * np.prod([(c[nu] + 2) / 3 for nu in range(4) if nu != mu]) for mu in range(4)])
    M = 2 - np.prod(c + 1) / 8 + m0
    X = M * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        X = X + 1j * pt[mu] * oracle.gamma(mu)
    return X, float(pt @ pt + M * M)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 6, 4, 8)])
def test_free_field_overlap(L):
    rho, n = 1.0, 8
    W = oracle.links(L, synth.unit_links(L))
    rng = np.random.default_rng(17)
    for _ in range(4):
        p = 2 * np.pi * np.array([rng.integers(0, L[mu]) for mu in range(4)]) / np.asarray(L)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        X, t = _free_symbol(p, -rho)
        want_sym = rho * (np.eye(4) + X * kl.r_diag_f64(t, n))
        got, _, _ = oracle.ov_apply(L, W, rho, n, plane_wave(L, p, u), tol=1e-14)
        want = plane_wave(L, p, want_sym @ u)
        assert np.abs(got - want).max() < 1e-12
        # and the exact free overlap rho [1 + X / sqrt(X^dag X)] within the KL bound
        exact = rho * (np.eye(4) + X / np.sqrt(t))
        x = np.sqrt(t)
        bound = abs(x * kl.r_diag_f64(t, n) - 1)
        assert np.abs(want_sym - exact).max() <= bound * np.abs(X).max() / x + 1e-15
