"""Pins of the oracle's link force and overlap gradient (Sec. 9).

The force is the derivative with respect to the Gell-Mann components of log U,
U_mu(z) -> exp(i omega^a lambda_a / 2) U_mu(z).  The oracle computes it by the
product rule along every shortest path of every off-axis link (App. C.1); the
pins differentiate numerically what the oracle's forward operator computes:

  * Brillouin operator: five-point central differences of
    S = Re sum_p w_p u_p^dag D v_p built from scratch (links by path averages,
    direct 81-term sum) for a spread of links, including the t-boundary links
    where the antiperiodic sign enters;
  * overlap operator: five-point central differences of
    S = Re chi^dag D_ov psi with D_ov from the dense eigendecomposition of
    H = gamma5 D(-rho) (same rational, no Krylov solver), against the oracle's
    formula built on CG shift solutions;
  * spinor gradient: D_ov^dag chi against the conjugate transpose of the dense
    overlap matrix;
  * the Gell-Mann matrices: hermitian, traceless, tr(lambda_a lambda_b) = 2 delta_ab
    and the su(3) structure constants f_123 = 1, f_458 = sqrt(3)/2.
"""

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth
from oracle import dense as odense


def _rand_spinor(rng, V):
    return rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))


def _fd5(S, U, mu, z, a, h):
    lam = oracle.gell_mann(a)
    vals = []
    for t in (2, 1, -1, -2):
        Ut = U.copy()
        Ut[mu, z] = sl.expm(1j * t * h * lam / 2) @ U[mu, z]
        vals.append(S(Ut))
    return (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)


def _samples(L, rng, count):
    """(mu, z, a) triples: boundary t links first, then random ones."""
    V = int(np.prod(L))
    per_t = V // L[3]
    out = [(3, V - 1, 0), (3, V - per_t, 1), (3, 0, 7), (3, per_t - 1, 4)]
    while len(out) < count:
        out.append((int(rng.integers(4)), int(rng.integers(V)), int(rng.integers(8))))
    return out


def test_gell_mann_algebra():
    lam = [oracle.gell_mann(a) for a in range(8)]
    for a in range(8):
        assert np.allclose(lam[a], lam[a].conj().T, atol=0)
        assert abs(np.trace(lam[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(lam[a] @ lam[b]) - 2.0 * (a == b)) < 1e-14
    # [lambda_a, lambda_b] = 2 i f_abc lambda_c
    def f(a, b, c):
        comm = lam[a] @ lam[b] - lam[b] @ lam[a]
        return (np.trace(comm @ lam[c]) / 4j).real
    assert abs(f(0, 1, 2) - 1.0) < 1e-14
    assert abs(f(3, 4, 7) - np.sqrt(3) / 2) < 1e-14
    assert abs(f(0, 3, 6) - 0.5) < 1e-14
    assert abs(f(0, 2, 3)) < 1e-14


@pytest.mark.parametrize("tbc", [0, 1])
def test_link_force_matches_finite_differences(tbc):
    L = (3, 3, 3, 4)
    V = int(np.prod(L))
    U = synth.random_links(L, 0.4, 5)
    rng = np.random.default_rng(11 + tbc)
    pairs = [(0.7, _rand_spinor(rng, V), _rand_spinor(rng, V)), (-1.3, _rand_spinor(rng, V), _rand_spinor(rng, V))]
    F = oracle.link_force(L, U, tbc, pairs)

    def S(Uw):
        W = oracle.links(L, Uw, tbc)
        return sum(w * np.vdot(u, oracle.dirac(L, W, 0.3, v)).real for w, u, v in pairs)

    scale = np.abs(F).max()
    for mu, z, a in _samples(L, rng, 12):
        fd = _fd5(S, U, mu, z, a, 1e-3)
        assert abs(fd - F[mu, z, a]) <= 1e-9 * scale, (mu, z, a, fd, F[mu, z, a])


def test_link_force_single_hop_closed_form():
    """Unit links, u = delta at x in (spin s, colour a'), v = delta at y = x + e_mu in
    (spin t, colour b), extent 3: the only displacement from x to y is d = e_mu, so
    S = Re (S_d)_{s t} W_d(x)_{a' b} and the force sits on U_mu(x) alone,
    F^a = Re[(S_d)_{s t} (i lambda_a / 2)_{a' b}]."""
    L = (3, 3, 3, 3)
    V = 81
    U = synth.unit_links(L)
    x = 13
    mu = 1
    c = [x % 3, (x // 3) % 3, (x // 9) % 3, x // 27]
    c[mu] = (c[mu] + 1) % 3
    y = c[0] + 3 * (c[1] + 3 * (c[2] + 3 * c[3]))
    s, ca, t, cb = 0, 2, 3, 1
    u = np.zeros((V, 4, 3), complex)
    v = np.zeros((V, 4, 3), complex)
    u[x, s, ca] = 1.0
    v[y, t, cb] = 1.0
    F = oracle.link_force(L, U, 0, [(1.0, u, v)])
    j = 40 + 3 ** mu
    Sd = oracle.spin_matrix(j, 0.0)
    for a in range(8):
        lam = oracle.gell_mann(a)
        expect = (Sd[s, t] * 0.5j * lam[ca, cb]).real
        assert abs(F[mu, x, a] - expect) < 1e-15
    F[mu, x] = 0.0
    assert np.abs(F).max() < 1e-15


def test_overlap_force_matches_dense_finite_differences():
    L = (2, 2, 3, 4)
    V = int(np.prod(L))
    rho, n = 1.0, 4
    U = synth.random_links(L, 0.3, 9)
    rng = np.random.default_rng(3)
    chi = _rand_spinor(rng, V)
    psi = _rand_spinor(rng, V)
    F, gpsi = oracle.ov_force(L, U, 1, rho, n, chi, psi, tol=1e-14)

    def dov(Uw):
        W = oracle.links(L, Uw, 1)
        D = oracle.dense_matrix(L, W, -rho)
        return odense.DenseOverlap(D, V, rho)

    def S(Uw):
        return np.vdot(chi.ravel(), dov(Uw).ov_apply(n, psi.ravel())).real

    scale = np.abs(F).max()
    for mu, z, a in _samples(L, rng, 8):
        fd = _fd5(S, U, mu, z, a, 1e-3)
        assert abs(fd - F[mu, z, a]) <= 1e-8 * scale, (mu, z, a, fd, F[mu, z, a])

    # spinor gradient: D_ov^dag chi from the dense matrix
    d = dov(U)
    G = d.fn_of_H(lambda lam: lam * oracle.kl.r_diag_f64(lam * lam, n))
    Dov = rho * (np.eye(12 * V) + d.G5[:, None] * G)
    ref = Dov.conj().T @ chi.ravel()
    assert np.linalg.norm(gpsi.ravel() - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("tbc", [0, 1])
def test_wilson_link_force_matches_finite_differences(tbc):
    """The Wilson force (the two hops every link enters) against five-point differences of
    Re sum_p w_p u_p^dag D_wil v_p, t-boundary links included."""
    L = (3, 3, 3, 4)
    V = int(np.prod(L))
    U = synth.random_links(L, 0.5, 41 + tbc)
    rng = np.random.default_rng(17 + tbc)
    pairs = [(0.7, _rand_spinor(rng, V), _rand_spinor(rng, V)), (-1.3, _rand_spinor(rng, V), _rand_spinor(rng, V))]
    m0 = -1.0
    F = oracle.link_force(L, U, tbc, pairs, kernel="wil")

    def S(Uw):
        K = oracle.WilsonKernel(Uw, tbc)
        return sum(w * np.vdot(u.ravel(), oracle.dirac(L, K, m0, v).ravel()).real for w, u, v in pairs)

    scale = np.abs(F).max()
    for mu, z, a in _samples(L, rng, 10):
        fd = _fd5(S, U, mu, z, a, 1e-3)
        assert abs(fd - F[mu, z, a]) <= 1e-9 * scale, (mu, z, a, fd, F[mu, z, a])


def test_wilson_overlap_force_matches_dense_finite_differences():
    L = (2, 2, 3, 4)
    V = int(np.prod(L))
    rho, n = 1.0, 4
    U = synth.random_links(L, 0.3, 29)
    rng = np.random.default_rng(23)
    chi = _rand_spinor(rng, V)
    psi = _rand_spinor(rng, V)
    F, gpsi = oracle.ov_force(L, U, 1, rho, n, chi, psi, tol=1e-14, kernel="wil")

    def dov(Uw):
        return odense.DenseOverlap(oracle.dense_matrix(L, oracle.WilsonKernel(Uw, 1), -rho), V, rho)

    def S(Uw):
        return np.vdot(chi.ravel(), dov(Uw).ov_apply(n, psi.ravel())).real

    scale = np.abs(F).max()
    for mu, z, a in _samples(L, rng, 6):
        fd = _fd5(S, U, mu, z, a, 1e-3)
        assert abs(fd - F[mu, z, a]) <= 1e-8 * scale, (mu, z, a, fd, F[mu, z, a])
    d = dov(U)
    G = d.fn_of_H(lambda lam: lam * oracle.kl.r_diag_f64(lam * lam, n))
    Dov = rho * (np.eye(12 * V) + d.G5[:, None] * G)
    assert np.linalg.norm(gpsi.ravel() - Dov.conj().T @ chi.ravel()) <= 1e-11 * np.linalg.norm(gpsi)
