"""Pins of the oracle's Kenney-Laub coefficients against the paper's printed
tables and against closed forms of the principal Pade functions (Sec. 3)."""

import os

import mpmath as mp
import numpy as np
import pytest

from oracle import kl
from tests.conftest import GOLDEN


def _half_ulp_printed(text: str) -> float:
    """Half a unit in the last printed digit of a decimal string."""
    mant = text.lower().split("e")[0]
    exp = int(text.lower().split("e")[1]) if "e" in text.lower() else 0
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (exp - decimals)


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


@mp.workdps(50)
def test_tab5_diagonal_partial_fractions():
    rows = _rows("kl_tab5.txt")
    by_n = {}
    for n, cn, cd, om, sg in rows:
        by_n.setdefault(int(n), []).append((int(cn), int(cd), om, sg))
    assert sorted(by_n) == [1, 2, 3, 4, 5, 6, 13]
    for n, poles in by_n.items():
        c0, om, sg = kl.kl_diag_coeffs(n)
        assert len(om) == len(poles) == n
        assert abs(c0 * poles[0][1] - poles[0][0]) < mp.mpf("1e-40")
        got = sorted(zip(sg, om))
        for (s, o), (cn, cd, om_p, sg_p) in zip(got, sorted(poles, key=lambda r: float(r[3]))):
            # the printed value is the exact one rounded to its last printed digit
            assert abs(o - mp.mpf(om_p)) <= _half_ulp_printed(om_p) * (1 + 1e-9), (n, om_p, o)
            assert abs(s - mp.mpf(sg_p)) <= _half_ulp_printed(sg_p) * (1 + 1e-9), (n, sg_p, s)


@mp.workdps(50)
def test_tab6_upper_diagonal_partial_fractions():
    rows = _rows("kl_tab6.txt")
    by_n = {}
    for n, om, sg in rows:
        by_n.setdefault(int(n), []).append((om, sg))
    assert sorted(by_n) == [1, 2, 3]
    for n, poles in by_n.items():
        om, sg = kl.kl_upper_coeffs(n)
        got = sorted(zip(sg, om))
        for (s, o), (om_p, sg_p) in zip(got, sorted(poles, key=lambda r: float(r[1]))):
            # One printed entry (n = 3, omega = 4.976067743425180) differs from the
            # exact 1/(3 cos^2(5 pi/12)) by 2.1e-15 relative, i.e. the table carries
            # its own double-precision evaluation error; allow 4e-15 relative.
            tol_o = max(_half_ulp_printed(om_p) * (1 + 1e-9), 4e-15 * abs(o))
            tol_s = max(_half_ulp_printed(sg_p) * (1 + 1e-9), 4e-15 * abs(s))
            assert abs(o - mp.mpf(om_p)) <= tol_o, (n, om_p, o)
            assert abs(s - mp.mpf(sg_p)) <= tol_s, (n, sg_p, s)


def _poly(coeffs, t):
    return mp.fsum(mp.mpf(c) * t**i for i, c in enumerate(coeffs))


@pytest.mark.parametrize("x", ["0.003", "0.05", "0.4", "0.99", "1", "1.7", "12", "300"])
def test_tab1_tab2_polynomial_forms(x):
    with mp.workdps(60):
        x = mp.mpf(x)
        for ln in _rows("kl_polynomials.txt"):
            s = " ".join(ln)
            mn, num, den = (p.split() for p in s.split("|"))
            m, n = int(mn[0]), int(mn[1])
            ref = x * _poly(num, x * x) / _poly(den, x * x)
            if m == n:
                got = kl.g_diag(x, n, dps=60)
            else:
                assert n == m + 1
                got = kl.g_upper(x, n, dps=60)
            assert abs(got - ref) <= mp.mpf("1e-45") * abs(ref)


@pytest.mark.parametrize("ell", [2, 3, 4, 5, 9, 17, 27, 33])
def test_binomial_and_tanh_forms(ell):
    """eq. (def_gell): g_l = ((1+x)^l - (1-x)^l)/((1+x)^l + (1-x)^l) = tanh(l artanh x)."""
    with mp.workdps(60):
        for x in ["0.01", "0.3", "0.8", "0.999"]:
            x = mp.mpf(x)
            binom = ((1 + x) ** ell - (1 - x) ** ell) / ((1 + x) ** ell + (1 - x) ** ell)
            th = mp.tanh(ell * mp.atanh(x))
            got = kl.g_diag(x, (ell - 1) // 2, dps=60) if ell % 2 else kl.g_upper(x, ell // 2, dps=60)
            assert abs(got - binom) <= mp.mpf("1e-45") * abs(binom)
            assert abs(got - th) <= mp.mpf("1e-45") * abs(th)
        for x in ["2.5", "40"]:  # beyond 1 only the binomial form applies
            x = mp.mpf(x)
            binom = ((1 + x) ** ell - (1 - x) ** ell) / ((1 + x) ** ell + (1 - x) ** ell)
            got = kl.g_diag(x, (ell - 1) // 2, dps=60) if ell % 2 else kl.g_upper(x, ell // 2, dps=60)
            assert abs(got - binom) <= mp.mpf("1e-45") * abs(binom)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_inversion_symmetry(n):
    """eq. (pade_symmetry): g_{2n+1}(1/x) = 1/g_{2n+1}(x), g_{2n}(1/x) = g_{2n}(x)."""
    with mp.workdps(50):
        for x in ["0.02", "0.5", "3", "77"]:
            x = mp.mpf(x)
            assert abs(kl.g_diag(1 / x, n) * kl.g_diag(x, n) - 1) < mp.mpf("1e-40")
            assert abs(kl.g_upper(1 / x, n) - kl.g_upper(x, n)) < mp.mpf("1e-40")


def test_nesting():
    """eq. (nesting): g_l'(g_l''(x)) = g_{l'l''}(x); e.g. f11 o f11 = f44, f11^(3) = f13,13, f22^(2) = f12,12."""
    with mp.workdps(60):
        for x in ["0.003", "0.2", "1.3", "50"]:
            x = mp.mpf(x)
            g3 = lambda v: kl.g_diag(v, 1, dps=60)  # noqa: E731
            g5 = lambda v: kl.g_diag(v, 2, dps=60)  # noqa: E731
            assert abs(g3(g3(x)) - kl.g_diag(x, 4, dps=60)) < mp.mpf("1e-45")
            assert abs(g3(g3(g3(x))) - kl.g_diag(x, 13, dps=60)) < mp.mpf("1e-45")
            assert abs(g5(g5(x)) - kl.g_diag(x, 12, dps=60)) < mp.mpf("1e-45")
            # [16/16] = g_33 = g_3 o g_11 (no printed table covers n = 16)
            assert abs(g3(kl.g_diag(x, 5, dps=60)) - kl.g_diag(x, 16, dps=60)) < mp.mpf("1e-45")


@mp.workdps(50)
def test_low_order_closed_forms():
    """eqs. (KL11_parfrac), (KL22_parfrac): sqrt(5) closed forms of n = 1, 2."""
    c0, om, sg = kl.kl_diag_coeffs(1)
    assert abs(om[0] - mp.mpf(8) / 9) < 1e-40 and abs(sg[0] - mp.mpf(1) / 3) < 1e-40  # (8/3)/3
    c0, om, sg = kl.kl_diag_coeffs(2)
    s5 = mp.sqrt(5)
    want = sorted([(1 - 2 / s5, 4 * (1 - 1 / s5) / 5), (1 + 2 / s5, 4 * (1 + 1 / s5) / 5)])
    got = sorted(zip(sg, om))
    for (s, o), (ws, wo) in zip(got, want):
        assert abs(s - ws) < 1e-40 and abs(o - wo) < 1e-40


def test_wouldbe_zero_mode_table():
    """Tab. wouldbe: 1 + f_nn^(k)(0.2 - 1) printed to two digits; closed form 2/(1 + 9^l), l = (2n+1)^k."""
    with mp.workdps(80):
        for k, n, val in _rows("kl_wouldbe.txt"):
            k, n = int(k), int(n)
            ell = (2 * n + 1) ** k
            closed = 2 / (1 + mp.mpf(9) ** ell)
            # printed value agrees with the closed form to its two digits
            printed = mp.mpf(val)
            assert abs(closed / printed - 1) < mp.mpf("0.05"), (k, n, val, closed)
            if ell <= 13**2:
                # and the iterated partial fractions reproduce the closed form
                x = mp.mpf("-0.8")
                for _ in range(k):
                    x = kl.g_diag(x, n, dps=80 + 2 * int(ell * 0.96))
                assert abs((1 + x) / closed - 1) < mp.mpf("1e-20"), (k, n)


@pytest.mark.parametrize("ell", [3, 9, 17, 33])
def test_derivative_closed_form(ell):
    """g_l'(x) = 4 l (1-x^2)^{l-1} / [(1+x)^l + (1-x)^l]^2 (Sec. 9)."""
    n = (ell - 1) // 2
    with mp.workdps(50):
        for x in ["0.1", "0.9", "1.5", "6"]:
            x = mp.mpf(x)
            c0, om, sg = kl.kl_diag_coeffs(n, 50)
            # derivative of x (c0 + sum omega/(x^2 + sigma)) term by term
            num = c0 + mp.fsum(o * (s - x * x) / (x * x + s) ** 2 for o, s in zip(om, sg))
            closed = 4 * ell * (1 - x * x) ** (ell - 1) / ((1 + x) ** ell + (1 - x) ** ell) ** 2
            assert abs(num - closed) <= mp.mpf("1e-30") * (1 + abs(closed))
