"""Kenney-Laub rational sign approximations, evaluated in high precision.

TEST INFRASTRUCTURE ONLY (part of the oracle).

The diagonal Kenney-Laub iteration function f_{n,n} = g_{2n+1} in its partial
fraction form, eq. (KLnn_parfrac) of Sec. 3.3:

    g_{2n+1}(x) = x/(2n+1) * sum_{i=0}^{n} (2 - delta_{i,n}) /
                  (sin^2(theta_i) + cos^2(theta_i) x^2),
    theta_i = (2i+1) pi / (4n+2).

The i = n term has theta_n = pi/2 and is the constant 1/(2n+1); every other
term is rewritten as omega_i / (x^2 + sigma_i) with
omega_i = 2 / ((2n+1) cos^2 theta_i) and sigma_i = tan^2 theta_i, the form of
Tab. 5 (App. B).  The first upper diagonal g_{2n} (Sec. 3.3, the formula
after eq. (KLnn_parfrac); Tab. 6) has no constant term and
omega_i = 1 / (n cos^2 theta_i), theta_i = (2i+1) pi / (4n).

All arithmetic is done with mpmath at `DPS` decimal digits; `*_f64` helpers
round the result to IEEE double.
"""

from __future__ import annotations

import mpmath as mp

DPS = 50


def kl_diag_coeffs(n: int, dps: int = DPS):
    """(c0, [omega_i], [sigma_i]) of f_{n,n} = g_{2n+1}, as mpf, i = 0..n-1."""
    with mp.workdps(dps):
        c0 = mp.mpf(1) / (2 * n + 1)
        om, sg = [], []
        for i in range(n):
            th = (2 * i + 1) * mp.pi / (4 * n + 2)
            om.append(2 / ((2 * n + 1) * mp.cos(th) ** 2))
            sg.append(mp.tan(th) ** 2)
        return c0, om, sg


def kl_upper_coeffs(n: int, dps: int = DPS):
    """([omega_i], [sigma_i]) of f_{n-1,n} = g_{2n}, i = 0..n-1 (no constant term)."""
    with mp.workdps(dps):
        om, sg = [], []
        for i in range(n):
            th = (2 * i + 1) * mp.pi / (4 * n)
            om.append(1 / (n * mp.cos(th) ** 2))
            sg.append(mp.tan(th) ** 2)
        return om, sg


def kl_diag_coeffs_f64(n: int):
    c0, om, sg = kl_diag_coeffs(n)
    return float(c0), [float(v) for v in om], [float(v) for v in sg]


def g_diag(x, n: int, dps: int = DPS):
    """g_{2n+1}(x) from the partial fractions, in mpmath."""
    with mp.workdps(dps):
        x = mp.mpf(x) if not isinstance(x, mp.mpc) else x
        c0, om, sg = kl_diag_coeffs(n, dps)
        return x * (c0 + mp.fsum(o / (x * x + s) for o, s in zip(om, sg)))


def g_upper(x, n: int, dps: int = DPS):
    """g_{2n}(x) from the partial fractions, in mpmath."""
    with mp.workdps(dps):
        x = mp.mpf(x)
        om, sg = kl_upper_coeffs(n, dps)
        return x * mp.fsum(o / (x * x + s) for o, s in zip(om, sg))


def r_diag_f64(t, n: int):
    """r_n(t) = c0 + sum_i omega_i / (t + sigma_i) in float64 (numpy-friendly), so
    that g_{2n+1}(x) = x r_n(x^2)."""
    c0, om, sg = kl_diag_coeffs_f64(n)
    out = c0
    for o, s in zip(om, sg):
        out = out + o / (t + s)
    return out
