"""Massive overlap solve of the oracle (TEST INFRASTRUCTURE ONLY).

Sec. 4 (massive overlap action, complete version): the massive Dirac equation D_m x = b with
the complete definition of D_m (eq. (def_mass_complete)) is solved as
    (D_ov + mt) x = bt,   mt = m / (1 - m/(2 rho)),
    bt = [1 + (m/(2 rho)) (1 - D_ov/(2 rho))] b / (1 - m/(2 rho))        eq. (upshot_complete)
(lattice spacing a = 1).  The traditional definition (eq. (def_mass_traditional)) gives the
same mt with bt = (mt/m) b (eq. (upshot_traditional)).  Sec. 7 solves it with BiCGstab as the
outer solver around the rational approximation of D_ov; `bicgstab` below is the textbook
method written out, with the oracle's own D_ov (per-shift CG) as the operator.

Sec. 8 (cascaded preconditioning) preconditions that outer solve by the same massive equation
with cheaper sign approximants: D^(0) = D_bri(-rho) = X, and D^(k) is D^(k-1) passed once more
through f_{1,1}, which by the nesting of the Kenney-Laub functions is X r_n(X^dag X) with
2n+1 = 3^k (n = 1, 4, 13, ...).  Every level solves A_k x = v with
A_k = rho [D^(k) + 1 + mt/rho] (= D_ov of order n_k plus mt), inverted approximately by
BiCGstab that is itself preconditioned by the next level.  The paper does not say how far the
preconditioner solves are taken; here each stops at a relative tolerance or an iteration cap
given per level.  `bicgstab_right` is the textbook right-preconditioned BiCGstab, in the form
that updates x with the preconditioned directions (so it tolerates a preconditioner that varies
from call to call).
"""

from __future__ import annotations

import numpy as np

from . import dirac, ov_apply


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


def bicgstab_right(apply, precond, b: np.ndarray, tol: float, maxit: int):
    """Right-preconditioned BiCGstab for apply(x) = b from x0 = 0, shadow residual r0 = b:
    the search directions p and s are passed through precond before the operator, and x is
    built from the preconditioned directions.  Returns (x, iterations, recursive rel. residual)."""
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
        ph = precond(p)
        v = apply(ph)
        alpha = rho_new / np.vdot(r0, v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bn:
            return x + alpha * ph, it, np.linalg.norm(s) / bn
        sh = precond(s)
        t = apply(sh)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho_new
        if np.linalg.norm(r) <= tol * bn:
            return x, it, np.linalg.norm(r) / bn
    return x, maxit, np.linalg.norm(r) / bn


def level_operator(L, W, rho: float, n_k: int, mt: float, ms_tol: float):
    """v -> A_k v = rho [D^(k) + 1 + mt/rho] v: the overlap approximant of Kenney-Laub order
    n_k plus mt (n_k > 0), or rho D_bri(-rho) v + (rho + mt) v for the Brillouin level (n_k = 0)."""
    if n_k == 0:
        return lambda v: rho * dirac(L, W, -rho, v) + (rho + mt) * v

    def A(v):
        Dv, _, _ = ov_apply(L, W, rho, n_k, v, ms_tol)
        return Dv + mt * v

    return A


def ov_solve_cascade(L, W, rho: float, n: int, m: float, b: np.ndarray, levels, complete: bool = True,
                     tol: float = 1e-10, maxit: int = 1000, inner_tol: float = 1e-13):
    """The massive solve of `ov_solve` with the outer BiCGstab right-preconditioned by the
    cascade `levels` = [(n_k, tol_k, maxit_k, ms_tol_k), ...] (levels[0] preconditions the
    outer operator, levels[k+1] preconditions levels[k]; n_k = 0, the Brillouin operator, only
    last).  Returns (x, outer iterations, true relative residual, iterations summed per level)."""
    mt = mass_tilde(m, rho)
    bt = rhs_tilde(L, W, rho, n, m, b, complete, inner_tol)
    counts = [0] * len(levels)

    def make_precond(k):
        if k >= len(levels):
            return lambda v: v
        n_k, tol_k, maxit_k, ms_tol_k = levels[k]
        A_k = level_operator(L, W, rho, n_k, mt, ms_tol_k)
        inner = make_precond(k + 1)

        def K(v):
            y, it, _ = bicgstab_right(A_k, inner, v, tol_k, maxit_k)
            counts[k] += it
            return y

        return K

    A = level_operator(L, W, rho, n, mt, inner_tol)
    x, it, _ = bicgstab_right(A, make_precond(0), bt, tol, maxit)
    res = np.linalg.norm(A(x) - bt) / np.linalg.norm(bt)
    return x, it, res, counts
