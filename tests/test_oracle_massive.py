"""Pins of the oracle's massive overlap solve (Sec. 4, complete and traditional versions;
BiCGstab outer solver of Sec. 7).

  * against a dense solve of (D_ov + mt) x = bt on 4^4 (D_ov from the eigendecomposition of
    H = gamma5 D(-rho), same rational, no Krylov solver);
  * the solution satisfies the complete massive equation D_m x = b with D_m written out as in
    the first form of eq. (def_mass_complete) (numerator times the inverse of the commuting
    denominator), which fixes mt and bt of eq. (upshot_complete) independently of how they are
    coded;
  * the contact-term identity S_com - S_tra = I/(2 rho) of eq. (contact), once with dense
    matrices and once with the two iterative solves: x_com - (1 - D_ov/(2 rho)) x_tra = b/(2 rho);
  * m -> 0 leaves the massless equation (mt = 0, bt = b).
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import dense as odense
from oracle import kl
from oracle import massive

L4 = (4, 4, 4, 4)
RHO, N, M = 1.0, 8, 0.3


@pytest.fixture(scope="module")
def setup():
    U = synth.random_links(L4, 0.3, synth.LINK_SEED_BASE + 1)
    W = oracle.links(L4, U)
    dov = odense.DenseOverlap(oracle.dense_matrix(L4, W, -RHO), 256, RHO)
    G = dov.fn_of_H(lambda lam: lam * kl.r_diag_f64(lam * lam, N))
    D = RHO * (np.eye(3072) + dov.G5[:, None] * G)
    b = synth.gaussian_source(L4, synth.SOURCE_SEED_BASE + 4)[0]
    return W, D, b


def test_mass_tilde():
    assert massive.mass_tilde(0.0, 1.0) == 0.0
    assert abs(massive.mass_tilde(0.5, 1.0) - 0.5 / 0.75) < 1e-15
    assert abs(massive.mass_tilde(0.2, 0.6) - 0.2 / (1 - 0.2 / 1.2)) < 1e-15


def test_complete_solve_against_dense(setup):
    W, D, b = setup
    x, it, res = massive.ov_solve(L4, W, RHO, N, M, b, complete=True, tol=1e-11)
    assert res < 1e-10 and it > 3
    mt = massive.mass_tilde(M, RHO)
    bv = b.ravel()
    bt = ((1 + M / (2 * RHO)) * bv - (M / (4 * RHO**2)) * (D @ bv)) / (1 - M / (2 * RHO))
    xd = np.linalg.solve(D + mt * np.eye(3072), bt)
    assert np.linalg.norm(x.ravel() - xd) <= 1e-9 * np.linalg.norm(xd)
    # D_m^com x = b with D_m^com = [D + m (1 - D/2rho)] [1 + (m/2rho)(1 - D/2rho)]^{-1}, the first
    # form of eq. (def_mass_complete) (its expanded second form prints m/(2 rho^2) for the D term of
    # the denominator where expanding the first gives m/(4 rho^2); the first form is the one that
    # eq. (upshot_complete) follows from)
    I = np.eye(3072)
    num = D + M * (I - D / (2 * RHO))
    den = I + (M / (2 * RHO)) * (I - D / (2 * RHO))
    Dm = num @ np.linalg.inv(den)
    assert np.linalg.norm(Dm @ xd - bv) <= 1e-11 * np.linalg.norm(bv)


def test_contact_term(setup):
    W, D, b = setup
    I = np.eye(3072)
    K = D + M * (I - D / (2 * RHO))
    Kinv = np.linalg.inv(K)
    S_tra = (I - D / (2 * RHO)) @ Kinv
    S_com = (I + (M / (2 * RHO)) * (I - D / (2 * RHO))) @ Kinv
    assert np.abs(S_com - S_tra - I / (2 * RHO)).max() < 1e-12
    # the same through the two iterative solves
    xc, _, _ = massive.ov_solve(L4, W, RHO, N, M, b, complete=True, tol=1e-12)
    xt, _, _ = massive.ov_solve(L4, W, RHO, N, M, b, complete=False, tol=1e-12)
    Dxt, _, _ = oracle.ov_apply(L4, W, RHO, N, xt, tol=1e-13)
    lhs = xc - (xt - Dxt / (2 * RHO))
    assert np.linalg.norm(lhs - b / (2 * RHO)) <= 1e-10 * np.linalg.norm(b)


def test_massless_limit(setup):
    W, D, b = setup
    assert massive.mass_tilde(0.0, RHO) == 0.0
    bt = massive.rhs_tilde(L4, W, RHO, N, 0.0, b, complete=True)
    assert np.array_equal(bt, b)
