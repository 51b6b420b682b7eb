"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws* inputs: random SU(3) gauge links, APE-smeared links,
point and Gaussian sources, random gauge transformations.  It contains none of
the arithmetic of the Brillouin operator, of the off-axis links, of the
Kenney-Laub sign function or of the overlap operator, so that the oracle and
the HIP library can both consume it without sharing any of the method.

Conventions (fixed for both sides):
  * lattice extents L = (Lx, Ly, Lz, Lt), direction mu = 0..3 <-> x, y, z, t;
  * site index s = x + Lx*(y + Ly*(z + Lz*t));
  * links   U[mu, s, a, b]      complex128, shape (4, V, 3, 3);
  * spinors psi[r, s, spin, c]  complex128, shape (nrhs, V, 4, 3).

The paper smears its gauge fields with APE steps but never writes the step
down; the standard form is used here:
  V_mu(x) = P_SU3[(1 - alpha) U_mu(x) + alpha/6 * sum of the 6 staples],
with P_SU3 the polar (unitary) factor divided by the cube root of its
determinant.  Seeds are numpy PCG64.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "gell_mann",
    "random_hermitian_traceless",
    "random_su3",
    "unit_links",
    "random_links",
    "ape_smear",
    "smeared_links",
    "point_source",
    "point_sources_12",
    "gaussian_source",
    "LINK_SEED_BASE",
    "SOURCE_SEED_BASE",
]

LINK_SEED_BASE = 1701
SOURCE_SEED_BASE = 726


def volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def random_hermitian_traceless(rng: np.random.Generator, n: int) -> np.ndarray:
    """A = sum_a xi_a lambda_a / 2 with xi_a ~ N(0, 1) i.i.d.; shape (n, 3, 3)."""
    xi = rng.standard_normal((n, 8))
    return np.einsum("na,aij->nij", xi, gell_mann() / 2)


def _expi_hermitian(A: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*A) for a batch of Hermitian 3x3 matrices (via eigh)."""
    w, Q = np.linalg.eigh(A)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", Q, ph, Q.conj())


def random_su3(n: int, eps: float, seed: int) -> np.ndarray:
    """n SU(3) matrices exp(i*eps*A), A Gaussian Hermitian traceless."""
    rng = np.random.default_rng(seed)
    return _expi_hermitian(random_hermitian_traceless(rng, n), eps)


def unit_links(L) -> np.ndarray:
    V = volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def random_links(L, eps: float, seed: int) -> np.ndarray:
    """Links U_mu(x) = exp(i*eps*A_mu(x)); shape (4, V, 3, 3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    A = random_hermitian_traceless(rng, 4 * V)
    return _expi_hermitian(A, eps).reshape(4, V, 3, 3)


def _shift(field: np.ndarray, L, mu: int, step: int) -> np.ndarray:
    """field(x + step*e_mu) for a site-indexed field of shape (V, ...), periodic."""
    Lx, Ly, Lz, Lt = L
    f = field.reshape((Lt, Lz, Ly, Lx) + field.shape[1:])
    axis = 3 - mu
    return np.roll(f, -step, axis=axis).reshape(field.shape)


def _project_su3(M: np.ndarray) -> np.ndarray:
    """Polar unitary factor of M, divided by the principal cube root of its det."""
    H = np.einsum("nji,njk->nik", M.conj(), M)
    w, Q = np.linalg.eigh(H)
    inv_sqrt = np.einsum("nij,nj,nkj->nik", Q, 1.0 / np.sqrt(w), Q.conj())
    W = M @ inv_sqrt
    det = np.linalg.det(W)
    return W / np.exp(1j * np.angle(det) / 3)[:, None, None]


def ape_smear(U: np.ndarray, L, alpha: float, steps: int) -> np.ndarray:
    """`steps` APE steps with staple weight alpha/6 (6 staples in 4D)."""
    U = U.copy()
    for _ in range(steps):
        new = np.empty_like(U)
        for mu in range(4):
            staple = np.zeros_like(U[mu])
            for nu in range(4):
                if nu == mu:
                    continue
                Unu = U[nu]
                Umu_xnu = _shift(U[mu], L, nu, +1)
                Unu_xmu = _shift(Unu, L, mu, +1)
                # forward staple U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
                staple += Unu @ Umu_xnu @ np.conj(np.swapaxes(Unu_xmu, -1, -2))
                # backward staple U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
                Unu_m = _shift(Unu, L, nu, -1)
                Umu_m = _shift(U[mu], L, nu, -1)
                Unu_mp = _shift(Unu_xmu, L, nu, -1)
                staple += np.conj(np.swapaxes(Unu_m, -1, -2)) @ Umu_m @ Unu_mp
            new[mu] = _project_su3((1 - alpha) * U[mu] + (alpha / 6) * staple)
        U = new
    return U


def smeared_links(L, eps: float, seed: int, ape_alpha: float = 0.6, ape_steps: int = 3) -> np.ndarray:
    """The link recipe of the larger workloads: exp(i*eps*A) then APE steps."""
    U = random_links(L, eps, seed)
    if ape_steps > 0:
        U = ape_smear(U, L, ape_alpha, ape_steps)
    return U


def point_source(L, spin: int = 0, colour: int = 0, site: int = 0) -> np.ndarray:
    """Unit point source; shape (1, V, 4, 3)."""
    psi = np.zeros((1, volume(L), 4, 3), dtype=np.complex128)
    psi[0, site, spin, colour] = 1
    return psi


def point_sources_12(L, site: int = 0) -> np.ndarray:
    """All 12 spin-colour point sources at one site; shape (12, V, 4, 3)."""
    psi = np.zeros((12, volume(L), 4, 3), dtype=np.complex128)
    for r in range(12):
        psi[r, site, r // 3, r % 3] = 1
    return psi


def gaussian_source(L, seed: int, nrhs: int = 1, normalize: bool = True) -> np.ndarray:
    """Complex Gaussian spinors (unit variance per component), optionally of unit norm."""
    rng = np.random.default_rng(seed)
    V = volume(L)
    psi = (rng.standard_normal((nrhs, V, 4, 3)) + 1j * rng.standard_normal((nrhs, V, 4, 3))) / np.sqrt(2)
    if normalize:
        psi /= np.linalg.norm(psi.reshape(nrhs, -1), axis=1)[:, None, None, None]
    return psi


# --------------------------------------------------------------- torch variant
# The same link recipe evaluated with torch on any device, for lattices where
# numpy would take minutes.  The Gaussian algebra elements are drawn by numpy
# with the same seed as `random_links`, so both variants agree to rounding.


def _t_dag(M):
    return M.conj().transpose(-1, -2).contiguous()


def _t_expi_hermitian(A, eps: float, squarings: int = 6, order: int = 12):
    """exp(i eps A) by a Taylor series of i eps A / 2^s followed by s squarings
    (matrix products only; |i eps A / 2^s| stays below 0.1 for these inputs)."""
    import torch

    X = (1j * eps / (1 << squarings)) * A
    eye = torch.eye(3, dtype=A.dtype, device=A.device).expand_as(A)
    E = eye.clone()
    term = eye.clone()
    for k in range(1, order + 1):
        term = (term @ X) / k
        E = E + term
    for _ in range(squarings):
        E = E @ E
    return E


def _t_inv3(M):
    """Inverse of a batch of 3x3 matrices by the adjugate."""
    import torch

    a = M
    c00 = a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1]
    c01 = a[..., 1, 2] * a[..., 2, 0] - a[..., 1, 0] * a[..., 2, 2]
    c02 = a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]
    c10 = a[..., 0, 2] * a[..., 2, 1] - a[..., 0, 1] * a[..., 2, 2]
    c11 = a[..., 0, 0] * a[..., 2, 2] - a[..., 0, 2] * a[..., 2, 0]
    c12 = a[..., 0, 1] * a[..., 2, 0] - a[..., 0, 0] * a[..., 2, 1]
    c20 = a[..., 0, 1] * a[..., 1, 2] - a[..., 0, 2] * a[..., 1, 1]
    c21 = a[..., 0, 2] * a[..., 1, 0] - a[..., 0, 0] * a[..., 1, 2]
    c22 = a[..., 0, 0] * a[..., 1, 1] - a[..., 0, 1] * a[..., 1, 0]
    det = a[..., 0, 0] * c00 + a[..., 0, 1] * c01 + a[..., 0, 2] * c02
    adj = torch.stack([torch.stack([c00, c10, c20], -1), torch.stack([c01, c11, c21], -1),
                       torch.stack([c02, c12, c22], -1)], -2)
    return adj / det.unsqueeze(-1).unsqueeze(-1), det


def _t_project_su3(M, iters: int = 12):
    """Polar unitary factor by the Newton iteration X <- (X + X^{-dag}) / 2 (matrix
    products and 3x3 inverses only), then divided by the cube root of its det."""
    import torch

    scale = torch.linalg.vector_norm(M, dim=(-2, -1)) / np.sqrt(3.0)
    X = M / scale.unsqueeze(-1).unsqueeze(-1)
    for _ in range(iters):
        Xi, _ = _t_inv3(X)
        X = 0.5 * (X + _t_dag(Xi))
    _, det = _t_inv3(X)
    return X / torch.exp(1j * torch.angle(det) / 3).unsqueeze(-1).unsqueeze(-1)


def _t_shift(field, L, mu: int, step: int):
    import torch

    Lx, Ly, Lz, Lt = L
    f = field.reshape((Lt, Lz, Ly, Lx) + tuple(field.shape[1:]))
    return torch.roll(f, shifts=-step, dims=3 - mu).reshape(field.shape)


def smeared_links_torch(L, eps: float, seed: int, ape_alpha: float = 0.6, ape_steps: int = 3, device="cuda",
                        chunk: int = 1 << 20):
    """`smeared_links` evaluated with torch on `device`; returns a (4, V, 3, 3)
    complex128 tensor on that device."""
    import torch

    V = volume(L)
    rng = np.random.default_rng(seed)
    lam = torch.from_numpy(gell_mann() / 2).to(device)
    U = torch.empty((4 * V, 3, 3), dtype=torch.complex128, device=device)
    for s in range(0, 4 * V, chunk):
        n = min(chunk, 4 * V - s)
        xi = torch.from_numpy(rng.standard_normal((n, 8))).to(device=device, dtype=torch.complex128)
        A = torch.einsum("na,aij->nij", xi, lam)
        U[s:s + n] = _t_expi_hermitian(A, eps)
    U = U.reshape(4, V, 3, 3)
    for _ in range(ape_steps):
        new = torch.empty_like(U)
        for mu in range(4):
            staple = torch.zeros_like(U[mu])
            for nu in range(4):
                if nu == mu:
                    continue
                Unu = U[nu]
                Umu_xnu = _t_shift(U[mu], L, nu, +1)
                Unu_xmu = _t_shift(Unu, L, mu, +1)
                staple += Unu @ Umu_xnu @ _t_dag(Unu_xmu)
                Unu_m = _t_shift(Unu, L, nu, -1)
                Umu_m = _t_shift(U[mu], L, nu, -1)
                Unu_mp = _t_shift(Unu_xmu, L, nu, -1)
                staple += _t_dag(Unu_m) @ Umu_m @ Unu_mp
            M = (1 - ape_alpha) * U[mu] + (ape_alpha / 6) * staple
            out = torch.empty_like(M)
            for s in range(0, V, chunk):
                out[s:s + chunk] = _t_project_su3(M[s:s + chunk])
            new[mu] = out
        U = new
    return U
