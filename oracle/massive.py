"""Massive overlap solve of the oracle (TEST INFRASTRUCTURE ONLY).

Sec. 4 (massive overlap action, complete version): the massive Dirac equation D_m x = b with
the complete definition of D_m (eq. (def_mass_complete)) is solved as
    (D_ov + mt) x = bt,   mt = m / (1 - m/(2 rho)),
    bt = [1 + (m/(2 rho)) (1 - D_ov/(2 rho))] b / (1 - m/(2 rho))        eq. (upshot_complete)
(lattice spacing a = 1).  The traditional definition (eq. (def_mass_traditional)) gives the
same mt with bt = (mt/m) b (eq. (upshot_traditional)).  Sec. 7 solves it with BiCGstab as the
outer solver around the rational approximation of D_ov; `bicgstab` below is the textbook
method written out, with the oracle's own D_ov (per-shift CG) as the operator.
"""

from __future__ import annotations

import numpy as np

from . import ov_apply


def mass_tilde(m: float, rho: float) -> float:
    """mt = m / (1 - m/(2 rho)), eq. (upshot_traditional) / (upshot_complete)."""
    return m / (1.0 - m / (2.0 * rho))


def rhs_tilde(L, W, rho: float, n: int, m: float, b: np.ndarray, complete: bool = True, tol: float = 1e-13):
    """bt of eq. (upshot_complete) (complete=True) or eq. (upshot_traditional)."""
    den = 1.0 - m / (2.0 * rho)
    if not complete:
        return b / den
    Db, _, _ = ov_apply(L, W, rho, n, b, tol)
    return ((1.0 + m / (2.0 * rho)) * b - (m / (4.0 * rho * rho)) * Db) / den


def bicgstab(apply, b: np.ndarray, tol: float, maxit: int):
    """Textbook BiCGstab for apply(x) = b from x0 = 0 with shadow residual r0 = b.
    Stops when the recursive residual is below tol |b|.  Returns (x, iterations, recursive rel. residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    r0 = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0, 0.0
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, maxit + 1):
        rho_new = np.vdot(r0, r)
        beta = (rho_new / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p)
        alpha = rho_new / np.vdot(r0, v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bn:
            x = x + alpha * p
            return x, it, np.linalg.norm(s) / bn
        t = apply(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho_new
        if np.linalg.norm(r) <= tol * bn:
            return x, it, np.linalg.norm(r) / bn
    return x, maxit, np.linalg.norm(r) / bn


def ov_solve(L, W, rho: float, n: int, m: float, b: np.ndarray, complete: bool = True, tol: float = 1e-10,
             maxit: int = 1000, inner_tol: float = 1e-13):
    """x with (D_ov + mt) x = bt for one right-hand side b of shape (V, 4, 3); returns
    (x, outer iterations, true relative residual of (D_ov + mt) x = bt)."""
    mt = mass_tilde(m, rho)
    bt = rhs_tilde(L, W, rho, n, m, b, complete, inner_tol)

    def A(v):
        Dv, _, _ = ov_apply(L, W, rho, n, v, inner_tol)
        return Dv + mt * v

    x, it, _ = bicgstab(A, bt, tol, maxit)
    res = np.linalg.norm(A(x) - bt) / np.linalg.norm(bt)
    return x, it, res
