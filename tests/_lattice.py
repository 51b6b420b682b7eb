"""Small lattice helpers for the tests (coordinates, shifts, plane waves).

These are geometry only: site numbering s = x + Lx*(y + Ly*(z + Lz*t)).
"""

import numpy as np


def coords(L):
    """(V, 4) integer coordinates of every site."""
    Lx, Ly, Lz, Lt = L
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


def site(L, c):
    c = np.asarray(c) % np.asarray(L)
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def shift_index(L, d):
    """Index array idx with field[idx] = field(x + d)."""
    return site(L, coords(L) + np.asarray(d))


def disp(j):
    """Displacement d of index j = sum_mu (d_mu + 1) 3^mu."""
    return np.array([(j // 3**mu) % 3 - 1 for mu in range(4)])


def plane_wave(L, p, u):
    """psi(x)_{s,c} = u_{s,c} exp(i p.x); u has shape (4, 3)."""
    ph = np.exp(1j * coords(L) @ np.asarray(p, dtype=np.float64))
    return ph[:, None, None] * u[None]
