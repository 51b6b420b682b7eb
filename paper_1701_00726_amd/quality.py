"""Operator-quality measures of Sec. 7, evaluated with the library's overlap apply on the GPU:

  * normality defect   |(D D^dag - D^dag D) eta|            (Sec. 7.1)
  * Ginsparg-Wilson defect |(D g5 + g5 D - D g5 D / rho) eta|  (Sec. 7.2, eq. (ginswils_one))
  * locality profile   |zeta(x)|, zeta = D eta for eta supported on the single site 0, against
                       the Euclidean distance |x| (minimal image), and the decay rate delta of
                       |zeta| ~ exp(-delta |x|)                          (Sec. 7.3)

D is any OverlapOp (kernel, c_SW, Kenney-Laub order and rho as built); D^dag is applied as
gamma5 D gamma5 (the overlap built from a gamma5-hermitian kernel is gamma5-hermitian).  Vector
norms and the gamma5 sign flips are plain tensor operations on the operator's outputs.
"""

from __future__ import annotations

import numpy as np

from . import _torch


def _g5(psi):
    torch = _torch()
    g = torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=psi.real.dtype, device=psi.device).view(1, 4, 1, 1)
    return psi * g


def _norms(v):
    torch = _torch()
    return torch.linalg.vector_norm(v.reshape(v.shape[0], -1), dim=1)


def normality_defect(op, eta):
    """|(D D^dag - D^dag D) eta| per column of eta (nrhs, 4, 3, V), D^dag = g5 D g5."""
    Ddag_eta, _ = op.apply(_g5(eta).contiguous())
    Ddag_eta = _g5(Ddag_eta)
    D_Ddag, _ = op.apply(Ddag_eta.contiguous())
    D_eta, _ = op.apply(eta)
    Ddag_D, _ = op.apply(_g5(D_eta).contiguous())
    Ddag_D = _g5(Ddag_D)
    return _norms(D_Ddag - Ddag_D).cpu().numpy()


def gw_defect(op, eta):
    """|(D g5 + g5 D - D g5 D / rho) eta| per column of eta."""
    rho = op.params.rho
    D_g5eta, _ = op.apply(_g5(eta).contiguous())
    D_eta, _ = op.apply(eta)
    D_g5D_eta, _ = op.apply(_g5(D_eta).contiguous())
    return _norms(D_g5eta + _g5(D_eta) - D_g5D_eta / rho).cpu().numpy()


def distances(L):
    """Euclidean minimal-image distance of every site from site 0 (site = x + Lx (y + Ly (z + Lz t)))."""
    L = np.asarray(L)
    V = int(np.prod(L))
    s = np.arange(V)
    r2 = np.zeros(V)
    for mu in range(4):
        c = s % L[mu]
        s = s // L[mu]
        d = np.minimum(c, L[mu] - c)
        r2 += d.astype(np.float64) ** 2
    return np.sqrt(r2)


def point_source(L, seed, device="cuda"):
    """A normalised Gaussian spin-colour vector on site 0 only, (1, 4, 3, V) complex128."""
    torch = _torch()
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    u /= np.linalg.norm(u)
    eta = np.zeros((1, 4, 3, V), dtype=np.complex128)
    eta[0, :, :, 0] = u
    return torch.from_numpy(eta).to(device)


def locality_profile(op, L, eta0):
    """(distances r, |zeta(x)| per site) for zeta = D eta0, eta0 supported on site 0."""
    zeta, _ = op.apply(eta0)
    mag = zeta[0].abs().pow(2).sum(dim=(0, 1)).sqrt().cpu().numpy()
    return distances(L), mag


def decay_rate(r, mag, rmin=2.0, rmax=None):
    """delta of |zeta| ~ exp(-delta r) from a least-squares line through log of the mean |zeta| at
    each distance in [rmin, rmax] (rmax: the largest distance present, less one)."""
    if rmax is None:
        rmax = r.max() - 1.0
    rs = np.unique(np.round(r, 9))
    rs = rs[(rs >= rmin) & (rs <= rmax)]
    means = np.array([mag[np.abs(r - x) < 1e-9].mean() for x in rs])
    keep = means > 0
    slope, _ = np.polyfit(rs[keep], np.log(means[keep]), 1)
    return -slope
