"""Pins of the oracle's off-axis links and Brillouin operator.

  * gamma basis: Clifford algebra, hermiticity, chiral form (App. C.1);
  * free field: plane waves against the momentum-space closed form (App. A);
  * the 15 doubler corners at 2 + m0 (Sec. 5);
  * off-axis links: unit field, hermitian reuse W_{-d}(x+d) = W_d(x)^dag
    (App. C.1), explicit two-path averages, the k-hop recursion, gauge
    covariance, antiperiodic sign;
  * operator: adjoint identity, gamma5-hermiticity (Sec. 4), gauge covariance,
    translation covariance.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from tests._lattice import coords, disp, plane_wave, shift_index, site


def test_gamma_basis():
    g = [oracle.gamma(mu) for mu in range(5)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * np.eye(4) * (a == b), atol=1e-15)
        # chiral representation: one entry of {+-1, +-i} per row and column
        nz = np.abs(g[a]) > 0
        assert (nz.sum(0) == 1).all() and (nz.sum(1) == 1).all()
        assert np.allclose(np.abs(g[a][nz]), 1)
    assert np.allclose(g[4], g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))  # chiral: gamma5 diagonal
    for a in range(4):
        assert np.allclose(g[4] @ g[a], -g[a] @ g[4])


def _free_symbol(p, m0):
    """Momentum-space Brillouin operator (App. A): i sum gamma_mu pt_mu + (1/2) pcheck^2 + m0."""
    p = np.asarray(p, dtype=np.float64)
    c, s = np.cos(p), np.sin(p)
    pt = np.array([s[mu] * np.prod([(c[nu] + 2) / 3 for nu in range(4) if nu != mu]) for mu in range(4)])
    half_pcheck2 = 2 - np.prod(c + 1) / 8
    D = (half_pcheck2 + m0) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        D = D + 1j * pt[mu] * oracle.gamma(mu)
    return D


@pytest.mark.parametrize("L,tbc", [((4, 4, 4, 4), 0), ((4, 6, 2, 8), 0), ((6, 4, 4, 6), 1)])
def test_free_field_plane_waves(L, tbc):
    V = int(np.prod(L))
    W = oracle.links(L, synth.unit_links(L), tbc=tbc)
    rng = np.random.default_rng(5)
    m0 = -0.73
    for trial in range(6):
        n = np.array([rng.integers(0, L[mu]) for mu in range(4)])
        p = 2 * np.pi * n / np.asarray(L)
        if tbc:
            p[3] = (2 * n[3] + 1) * np.pi / L[3]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = plane_wave(L, p, u)
        got = oracle.dirac(L, W, m0, psi)
        want = plane_wave(L, p, _free_symbol(p, m0) @ u)
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max(), (L, p)
        assert got.shape == (V, 4, 3)


def test_doublers_and_zero_mode():
    """At the 16 corners p in {0, pi}^4: D = m0 at p = 0 and D = 2 + m0 at the 15 others."""
    L = (4, 4, 4, 4)
    W = oracle.links(L, synth.unit_links(L))
    m0 = 0.0
    u = np.arange(12, dtype=np.complex128).reshape(4, 3) + 1
    for corner in itertools.product([0, 1], repeat=4):
        p = np.pi * np.asarray(corner)
        got = oracle.dirac(L, W, m0, plane_wave(L, p, u))
        lam = 0.0 if sum(corner) == 0 else 2.0
        assert np.abs(got - lam * plane_wave(L, p, u)).max() < 1e-13


def test_constant_field_laplacian_sums_to_zero():
    L = (4, 4, 4, 4)
    W = oracle.links(L, synth.unit_links(L))
    psi = np.ones((256, 4, 3), dtype=np.complex128)
    assert np.abs(oracle.dirac(L, W, 0.37, psi) - 0.37 * psi).max() < 1e-14


@pytest.fixture(scope="module")
def rough():
    L = (4, 4, 6, 4)
    U = synth.random_links(L, 0.8, 11)
    return L, U, oracle.links(L, U)


def test_unit_links_give_unit_W():
    L = (3, 4, 3, 4)
    W = oracle.links(L, synth.unit_links(L))
    assert np.abs(W - np.eye(3)).max() < 1e-15


def test_antiperiodic_sign():
    L = (4, 4, 4, 4)
    W = oracle.links(L, synth.unit_links(L), tbc=1)
    t = coords(L)[:, 3]
    for j in range(81):
        d = disp(j)
        crosses = (t + d[3] < 0) | (t + d[3] >= L[3])
        want = np.where(crosses, -1.0, 1.0)[:, None, None] * np.eye(3)
        assert np.abs(W[:, j] - want).max() < 1e-15


def test_hermitian_reuse(rough):
    """W_{-d}(x+d) = W_d(x)^dag, which is why only 40 of 80 links need storing (App. C.1)."""
    L, U, W = rough
    for j in range(81):
        idx = shift_index(L, disp(j))
        assert np.abs(W[idx, 80 - j] - np.conj(np.swapaxes(W[:, j], -1, -2))).max() < 1e-15


def test_one_and_two_hop_links(rough):
    L, U, W = rough
    dag = lambda M: np.conj(np.swapaxes(M, -1, -2))  # noqa: E731
    j_of = lambda d: int(sum((d[mu] + 1) * 3**mu for mu in range(4)))  # noqa: E731
    for mu in range(4):
        e = np.eye(4, dtype=int)[mu]
        assert np.abs(W[:, j_of(e)] - U[mu]).max() < 1e-15
        assert np.abs(W[:, j_of(-e)] - dag(U[mu][shift_index(L, -e)])).max() < 1e-15
    # two hops: the mean of the two paths, written out
    for mu, nu in [(0, 1), (1, 3), (0, 2)]:
        emu, enu = np.eye(4, dtype=int)[mu], np.eye(4, dtype=int)[nu]
        Umu, Unu = U[mu], U[nu]
        want = 0.5 * (Umu @ Unu[shift_index(L, emu)] + Unu @ Umu[shift_index(L, enu)])
        assert np.abs(W[:, j_of(emu + enu)] - want).max() < 1e-15
        # +mu then -nu:  U_mu(x) U_nu(x+mu-nu)^dag ;  -nu then +mu: U_nu(x-nu)^dag U_mu(x-nu)
        want = 0.5 * (
            Umu @ dag(Unu[shift_index(L, emu - enu)]) + dag(Unu[shift_index(L, -enu)]) @ Umu[shift_index(L, -enu)]
        )
        assert np.abs(W[:, j_of(emu - enu)] - want).max() < 1e-15


def test_k_hop_recursion(rough):
    """Averages over shortest paths obey W_d(x) = (1/k) sum_{mu in supp d} T_mu W_{d - s_mu e_mu}(x + s_mu e_mu)."""
    L, U, W = rough
    dag = lambda M: np.conj(np.swapaxes(M, -1, -2))  # noqa: E731
    for j in range(81):
        d = disp(j)
        supp = [mu for mu in range(4) if d[mu] != 0]
        k = len(supp)
        if k < 2:
            continue
        acc = 0
        for mu in supp:
            e = np.eye(4, dtype=int)[mu] * d[mu]
            T = U[mu] if d[mu] > 0 else dag(U[mu][shift_index(L, e)])
            jr = int(sum((d[nu] - e[nu] + 1) * 3**nu for nu in range(4)))
            acc = acc + T @ W[shift_index(L, e), jr]
        assert np.abs(W[:, j] - acc / k).max() < 1e-14


def _gauge(L, U, G):
    dag = lambda M: np.conj(np.swapaxes(M, -1, -2))  # noqa: E731
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = G @ U[mu] @ dag(G[shift_index(L, np.eye(4, dtype=int)[mu])])
    return Ug


def test_gauge_covariance(rough):
    L, U, W = rough
    V = int(np.prod(L))
    G = synth.random_su3(V, 2.0, 99)
    Wg = oracle.links(L, _gauge(L, U, G))
    dag = lambda M: np.conj(np.swapaxes(M, -1, -2))  # noqa: E731
    for j in range(81):
        want = G @ W[:, j] @ dag(G[shift_index(L, disp(j))])
        assert np.abs(Wg[:, j] - want).max() < 1e-14
    psi = synth.gaussian_source(L, 3)[0]
    m0 = -1.0
    lhs = oracle.dirac(L, Wg, m0, np.einsum("xab,xsb->xsa", G, psi))
    rhs = np.einsum("xab,xsb->xsa", G, oracle.dirac(L, W, m0, psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_adjoint_and_gamma5_hermiticity(rough):
    L, U, W = rough
    m0 = -1.0
    psi = synth.gaussian_source(L, 4)[0]
    phi = synth.gaussian_source(L, 5)[0]
    Dpsi = oracle.dirac(L, W, m0, psi)
    Dadj_phi = oracle.dirac_adj(L, W, m0, phi)
    assert abs(np.vdot(phi, Dpsi) - np.vdot(Dadj_phi, psi)) < 1e-14
    g5D_g5 = oracle.gamma5_apply(oracle.dirac(L, W, m0, oracle.gamma5_apply(phi)))
    assert np.abs(g5D_g5 - Dadj_phi).max() < 1e-14
    # without the k! average (one fixed path order) gamma5-hermiticity is lost
    Wbad = W.copy()
    for j in range(81):
        if np.count_nonzero(disp(j)) == 2:
            d = disp(j)
            mu, nu = [m for m in range(4) if d[m] != 0]
            if d[mu] > 0 and d[nu] > 0:
                e1, e2 = np.eye(4, dtype=int)[mu], np.eye(4, dtype=int)[nu]
                Wbad[:, j] = U[mu] @ U[nu][shift_index(L, e1)]
    bad = oracle.gamma5_apply(oracle.dirac(L, Wbad, m0, oracle.gamma5_apply(phi)))
    assert np.abs(bad - oracle.dirac_adj(L, Wbad, m0, phi)).max() > 1e-3


def test_translation_covariance(rough):
    L, U, W = rough
    a = np.array([1, 2, 0, 3])
    idx = shift_index(L, a)
    Ut = U[:, idx]
    Wt = oracle.links(L, Ut)
    psi = synth.gaussian_source(L, 6)[0]
    out = oracle.dirac(L, W, -1.0, psi)
    out_t = oracle.dirac(L, Wt, -1.0, psi[idx])
    assert np.abs(out_t - out[idx]).max() < 1e-14


def test_dense_matches_apply(rough):
    L, U, W = rough
    L = (2, 2, 2, 4)
    U = synth.random_links(L, 0.5, 12)
    W = oracle.links(L, U)
    M = oracle.dense_matrix(L, W, -0.9)
    psi = synth.gaussian_source(L, 7)[0]
    got = (M @ psi.reshape(-1)).reshape(psi.shape)
    assert np.abs(got - oracle.dirac(L, W, -0.9, psi)).max() < 1e-14
    assert site(L, np.array([1, 1, 1, 3])) == 1 + 2 * (1 + 2 * (1 + 2 * 3))


@pytest.mark.parametrize("tbc", [0, 1])
def test_sampled_site_operator_matches_full_sums(tbc):
    """dirac_at / dirac_adj_at (links built per sampled site) reproduce the full-lattice
    sums at those sites, including sites on every face of a non-cubic lattice."""
    L = (4, 4, 4, 6)
    V = 384
    U = synth.random_links(L, 0.5, 3)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    W = oracle.links(L, U, tbc)
    full, fadj = oracle.dirac(L, W, -0.7, psi), oracle.dirac_adj(L, W, -0.7, psi)
    sites = [0, 3, 15, 63, 64, 191, 320, 383] + list(rng.integers(0, V, 8))
    a = oracle.dirac_at(L, U, tbc, -0.7, psi, sites)
    b = oracle.dirac_adj_at(L, U, tbc, -0.7, psi, sites)
    scale = np.abs(full).max()
    assert np.abs(a - full[sites]).max() <= 1e-14 * scale
    assert np.abs(b - fadj[sites]).max() <= 1e-14 * scale
