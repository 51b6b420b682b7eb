"""Pins of the oracle's sign-approximation variants (Sec. 3.3, App. B):

  * the first upper diagonal g_{2n} = f_{n-1,n} in partial fractions (no constant term) against
    its closed form [(1+x)^{2n} - (1-x)^{2n}] / [(1+x)^{2n} + (1-x)^{2n}] applied through the
    dense eigendecomposition of H (no coefficients on that side), for the sign function and the
    overlap operator;
  * the overlap force with g_{2n} against five-point differences of that dense operator;
  * relaxed per-shift stopping (tol * omega_max / omega_i): every shift meets its own tolerance,
    the small shifts stop earlier, and the result stays within the error bound that the
    residuals imply (sum_i omega_i |r_i| / sigma_i, since X^dag X >= 0);
  * the result bound: |X (X^dag X + sigma)^{-1}| equals the largest s / (s^2 + sigma) over the
    singular values s of X, at most 1 / (2 sqrt(sigma)) and nearly that when sqrt(sigma) lies
    inside the singular spectrum (dense SVD); stopping the shifts so that
    sum_i omega_i |r_i| / (2 sqrt(sigma_i)) <= tol |b| keeps the sign function within tol |b| of
    the exact rational (dense eigendecomposition).
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import dense as odense
from tests.test_oracle_force import _fd5, _rand_spinor, _samples


def g_upper_closed(x, n):
    p, q = (1 + x) ** (2 * n), (1 - x) ** (2 * n)
    return (p - q) / (p + q)


def g_diag_closed(x, n):
    p, q = (1 + x) ** (2 * n + 1), (1 - x) ** (2 * n + 1)
    return (p - q) / (p + q)


L_SMALL = (2, 2, 4, 4)


@pytest.fixture(scope="module")
def small():
    U = synth.random_links(L_SMALL, 0.4, synth.LINK_SEED_BASE + 8)
    W = oracle.links(L_SMALL, U)
    V = int(np.prod(L_SMALL))
    d = odense.DenseOverlap(oracle.dense_matrix(L_SMALL, W, -1.0), V, 1.0)
    b = synth.gaussian_source(L_SMALL, synth.SOURCE_SEED_BASE + 8)[0]
    return W, d, b


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_upper_diagonal_sign_and_overlap_against_closed_form(small, n):
    W, d, b = small
    got, _, rel = oracle.sign_apply(L_SMALL, W, 1.0, n, b, tol=1e-14, kind="upper")
    want = d.apply_fn(lambda lam: g_upper_closed(lam, n), b.ravel()).reshape(b.shape)
    assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want)
    assert max(rel) <= 1e-13
    ov, _, _ = oracle.ov_apply(L_SMALL, W, 1.0, n, b, tol=1e-14, kind="upper")
    want_ov = b + (d.G5 * d.apply_fn(lambda lam: g_upper_closed(lam, n), b.ravel())).reshape(b.shape)
    assert np.linalg.norm(ov - want_ov) <= 1e-11 * np.linalg.norm(want_ov)
    # the diagonal member through the same closed form, for contrast: g_{2n+1} != g_{2n}
    gd, _, _ = oracle.sign_apply(L_SMALL, W, 1.0, n, b, tol=1e-14)
    want_d = d.apply_fn(lambda lam: g_diag_closed(lam, n), b.ravel()).reshape(b.shape)
    assert np.linalg.norm(gd - want_d) <= 1e-11 * np.linalg.norm(want_d)
    assert np.linalg.norm(gd - got) > 1e-6


def test_upper_diagonal_force_matches_dense_finite_differences():
    L = (2, 2, 3, 4)
    V = int(np.prod(L))
    rho, n = 1.0, 3
    U = synth.random_links(L, 0.3, 19)
    rng = np.random.default_rng(13)
    chi = _rand_spinor(rng, V)
    psi = _rand_spinor(rng, V)
    F, gpsi = oracle.ov_force(L, U, 0, rho, n, chi, psi, tol=1e-14, kind="upper")

    def dov(Uw):
        D = oracle.dense_matrix(L, oracle.links(L, Uw, 0), -rho)
        return odense.DenseOverlap(D, V, rho)

    def S(Uw):
        d = dov(Uw)
        v = psi.ravel()
        return np.vdot(chi.ravel(), rho * (v + d.G5 * d.apply_fn(lambda lam: g_upper_closed(lam, n), v))).real

    scale = np.abs(F).max()
    for mu, z, a in _samples(L, rng, 6):
        fd = _fd5(S, U, mu, z, a, 1e-3)
        assert abs(fd - F[mu, z, a]) <= 1e-8 * scale, (mu, z, a, fd, F[mu, z, a])
    d = dov(U)
    G = d.fn_of_H(lambda lam: g_upper_closed(lam, n))
    Dov = rho * (np.eye(12 * V) + d.G5[:, None] * G)
    ref = Dov.conj().T @ chi.ravel()
    assert np.linalg.norm(gpsi.ravel() - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["diag", "upper"])
def test_relaxed_shift_tolerances(small, kind):
    W, d, b = small
    n, tol = 6, 1e-9
    c0, om, sg = oracle.kl_coeffs(n, kind)
    y_strict, it_strict, _ = oracle.rational_apply(L_SMALL, W, -1.0, n, b, tol=tol, kind=kind)
    y_relax, it_relax, rel = oracle.rational_apply(L_SMALL, W, -1.0, n, b, tol=tol, kind=kind, relax=True)
    wmax = max(om)
    for i in range(n):
        assert rel[i] <= tol * wmax / om[i]
        assert it_relax[i] <= it_strict[i]
    assert it_relax[0] < it_strict[0]  # the smallest shift carries the smallest weight
    # exact r_n(A) b from the eigendecomposition of H (A = H^2)
    exact = d.apply_fn(lambda lam: c0 + sum(o / (lam * lam + s) for o, s in zip(om, sg)), b.ravel())
    bound = sum(o * tol * (wmax / o) / s for o, s in zip(om, sg)) * np.linalg.norm(b)
    err = np.linalg.norm(y_relax.ravel() - exact)
    assert err <= bound
    assert np.linalg.norm(y_strict.ravel() - exact) <= sum(o * tol / s for o, s in zip(om, sg)) * np.linalg.norm(b)


def test_result_bound_constant(small):
    W, d, b = small
    D = d.D
    sv = np.linalg.svd(D, compute_uv=False)
    A = D.conj().T @ D
    eye = np.eye(D.shape[0])
    _, _, sg = oracle.kl_coeffs(6)
    inside = 0
    for sig in sg:
        nrm = np.linalg.norm(D @ np.linalg.inv(A + sig * eye), 2)
        assert abs(nrm - np.max(sv / (sv * sv + sig))) <= 1e-10 * nrm
        assert nrm <= (1 + 1e-10) / (2.0 * np.sqrt(sig))
        if sv.min() <= np.sqrt(sig) <= sv.max():
            inside += 1
            assert nrm >= 0.95 / (2.0 * np.sqrt(sig)), (sig, nrm)
    assert inside >= 2


@pytest.mark.parametrize("kind", ["diag", "upper"])
def test_result_bound_stopping(small, kind):
    W, d, b = small
    n, tol = 6, 1e-8
    c0, om, sg = oracle.kl_coeffs(n, kind)
    got, it_b, rel = oracle.sign_apply(L_SMALL, W, 1.0, n, b, tol=tol, kind=kind, relax="bound")
    w = [o / (2.0 * np.sqrt(s)) for o, s in zip(om, sg)]
    assert sum(wi * r for wi, r in zip(w, rel)) <= tol * (1 + 1e-9)
    exact = d.apply_fn(lambda lam: lam * (c0 + sum(o / (lam * lam + s) for o, s in zip(om, sg))), b.ravel())
    err = np.linalg.norm(got.ravel() - exact)
    assert err <= tol * np.linalg.norm(b)
    # the bound is not slack by orders of magnitude: the error is within 1000x of it
    assert err >= 1e-3 * tol * np.linalg.norm(b)
