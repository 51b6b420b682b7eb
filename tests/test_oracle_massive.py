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


def test_nested_operators_are_the_kl_approximants():
    """Sec. 8 builds D^(1) = X (1/3 + (8/9)/(A + 1/3)) and D^(2), D^(3) by applying the same
    f_{1,1} to D^(1), D^(2) (with A^(k) = D^(k)dag D^(k)), and then writes D^(2) and D^(3) with the
    partial fractions of f_{4,4} and f_{13,13} in A = X^dag X.  Dense check on a small lattice:
    the nested matrices equal X r_n(A) with the oracle's coefficients for n = 1, 4, 13."""
    L = (2, 2, 4, 4)
    U = synth.random_links(L, 0.5, synth.LINK_SEED_BASE + 7)
    X = oracle.dense_matrix(L, oracle.links(L, U), -RHO)
    N_ = X.shape[0]
    I = np.eye(N_)

    def f11_step(D):
        A = D.conj().T @ D
        return D @ (I / 3 + (8.0 / 9.0) * np.linalg.inv(A + I / 3))

    def kl_matrix(n):
        c0, om, sg = kl.kl_diag_coeffs_f64(n)
        A = X.conj().T @ X
        R = c0 * I
        for o, s_ in zip(om, sg):
            R = R + o * np.linalg.inv(A + s_ * I)
        return X @ R

    D = X
    for n in (1, 4, 13):
        D = f11_step(D)
        K = kl_matrix(n)
        assert np.abs(D - K).max() <= 1e-11 * np.abs(K).max(), n


def test_cascaded_solve_matches_plain_solve(setup):
    """The preconditioned solves reach the solution of the unpreconditioned equation: f_{1,1}
    with the Brillouin operator as one-level preconditioner, f_{4,4} with two levels (f_{1,1},
    then Brillouin), as in Tab. cascaded; the preconditioned outer solves take fewer iterations."""
    W, _, b = setup
    for n, levels in ((1, [(0, 0.1, 30, 0.0)]), (4, [(1, 0.1, 30, 1e-8), (0, 0.1, 30, 0.0)])):
        x0, it0, res0 = massive.ov_solve(L4, W, RHO, n, M, b, complete=True, tol=1e-11)
        x1, it1, res1, counts = massive.ov_solve_cascade(L4, W, RHO, n, M, b, levels, complete=True, tol=1e-11)
        assert res0 < 1e-10 and res1 < 1e-10
        assert np.linalg.norm(x1 - x0) <= 1e-9 * np.linalg.norm(x0), n
        assert it1 < it0 and all(c > 0 for c in counts), (n, it0, it1, counts)
