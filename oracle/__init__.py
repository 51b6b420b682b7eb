"""FP64 CPU oracle for the Brillouin-kernel overlap operator (arXiv:1701.00726).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the HIP
library (`paper_1701_00726_amd`); the two meet only through the seeded inputs
of `synth`.

Layouts here are the oracle's own: links U (4, V, 3, 3), off-axis links
W (V, 81, 3, 3), spinors (nrhs, V, 4, 3), all complex128.  The heavy loops
are plain C with OpenMP (`oracle.c`, built on first import with gcc).

Functions and the passages they follow:
  links            off-axis links as averages over all shortest paths (App. C.1)
  dirac, dirac_adj Brillouin operator eq. (def_bril), c_SW = 0, and its adjoint
  dense_matrix     the same operator as a dense matrix (small lattices)
  dirac_at, dirac_adj_at  the same sums at listed sites only, links built on the fly from U
  cg               textbook CG on (D^dag D + sigma) x = b
  rational_apply   c0 b + sum_i omega_i (D^dag D + sigma_i)^{-1} b, eq. (KLnn_parfrac)
  sign_apply       gamma5 g_{2n+1}(H) b with H = gamma5 D(-rho), Sec. 3.3 / eq. (def_over)
  ov_apply         rho (1 + gamma5 g_{2n+1}(H)) b, eq. (def_over)
  link_force       dS/d omega for S = Re sum_p w_p u_p^dag D v_p, U -> exp(i omega^a
                   lambda_a / 2) U (Sec. 9: derivative with respect to the Gell-Mann
                   components of log U), product rule along every path of App. C.1
  massive.ov_solve (D_ov + mt) x = bt of the complete massive form (Sec. 4), by textbook BiCGstab
                   (Sec. 7) around ov_apply
  ov_force         the same derivative for S = Re chi^dag D_ov psi with the fixed-order
                   rational of eq. (KLnn_parfrac) inside eq. (def_over) (Sec. 9), and
                   the spinor gradient D_ov^dag chi
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import kl

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lock = threading.Lock()
_lib = None


def build(force: bool = False, sanitize_to: str | None = None) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP).  sanitize_to: instead build a copy
    instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (ROCm's clang, so that it
    shares the sanitizer runtime of the library's sanitized host code) at that path."""
    if sanitize_to:
        subprocess.check_call(
            ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             "-shared-libsan", "-o", sanitize_to, _SRC, "-lm"]
        )
        return sanitize_to
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            alt = os.environ.get("ORACLE_LIB")  # a separately built copy (the sanitizer job)
            if alt:
                lib = ctypes.CDLL(alt)
            else:
                build()
                lib = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            lib.orc_links.argtypes = [P, I, P, P]
            lib.orc_dirac.argtypes = [P, P, D, P, P, I]
            lib.orc_dirac_adj.argtypes = [P, P, D, P, P, I]
            lib.orc_dirac_dense.argtypes = [P, P, D, P]
            lib.orc_gamma.argtypes = [I, P]
            lib.orc_spin_matrix.argtypes = [I, D, P]
            lib.orc_wilson.argtypes = [P, I, P, D, P, P, I]
            lib.orc_wilson_adj.argtypes = [P, I, P, D, P, P, I]
            lib.orc_wilson_dense.argtypes = [P, I, P, D, P]
            lib.orc_clover.argtypes = [P, P, D, P]
            lib.orc_clover_apply.argtypes = [P, P, P, P, I, I]
            lib.orc_cg.argtypes = [P, I, I, P, P, D, D, P, P, D, I, P]
            lib.orc_cg.restype = I
            lib.orc_rational.argtypes = [P, I, I, P, P, D, I, D, P, P, P, P, D, I, P, P]
            lib.orc_rational.restype = I
            lib.orc_num_threads.restype = I
            lib.orc_lambda.argtypes = [I, P]
            lib.orc_dirac_at.argtypes = [P, I, P, D, P, I, P, P]
            lib.orc_dirac_adj_at.argtypes = [P, I, P, D, P, I, P, P]
            lib.orc_link_force.argtypes = [P, I, P, I, P, P, P, P]
            lib.orc_wilson_force.argtypes = [P, I, P, I, P, P, P, P]
            _lib = lib
    return _lib


def _geom(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().orc_num_threads())


def volume(L):
    return int(np.prod(L))


# --------------------------------------------------------------------------- basis


def gamma(mu: int) -> np.ndarray:
    """gamma_mu (mu = 0..3 for x, y, z, t) or gamma5 (mu = 4) of the oracle's chiral basis."""
    out = np.zeros(16, dtype=np.complex128)
    _load().orc_gamma(int(mu), _ptr(out))
    return out.reshape(4, 4)


def spin_matrix(j: int, m0: float) -> np.ndarray:
    """S_d for displacement index j = sum_mu (d_mu + 1) 3^mu."""
    out = np.zeros(16, dtype=np.complex128)
    _load().orc_spin_matrix(int(j), float(m0), _ptr(out))
    return out.reshape(4, 4)


def gamma5_apply(psi: np.ndarray) -> np.ndarray:
    g5 = gamma(4)
    return np.einsum("st,...tc->...sc", g5, psi)


# ------------------------------------------------------------------- operator


def links(L, U: np.ndarray, tbc: int = 0) -> np.ndarray:
    """Off-axis links W (V, 81, 3, 3) from links U (4, V, 3, 3); brute-force paths."""
    V = volume(L)
    U = _c128(U)
    assert U.shape == (4, V, 3, 3)
    W = np.zeros((V, 81, 3, 3), dtype=np.complex128)
    _load().orc_links(_ptr(_geom(L)), int(tbc), _ptr(U), _ptr(W))
    return W


class WilsonKernel:
    """The Wilson operator of eq. (def_wils) as the kernel: the gauge field U (4, V, 3, 3), the
    t boundary condition and optionally a clover field (V, 12, 12) from `clover_field`.
    Wherever the functions below take the Brillouin link array W, an instance of this class
    selects the Wilson operator instead."""

    def __init__(self, U: np.ndarray, tbc: int = 0, clover: np.ndarray | None = None):
        self.U = _c128(U)
        self.tbc = int(tbc)
        self.clover = None if clover is None else _c128(clover)


class BrillouinKernel:
    """The Brillouin operator with a clover term: the link array W of `links` and a clover field
    (V, 12, 12).  A bare W array is the Brillouin operator with c_SW = 0."""

    def __init__(self, W: np.ndarray, clover: np.ndarray | None = None):
        self.W = _c128(W)
        self.clover = None if clover is None else _c128(clover)


def _kernel_args(W):
    """(kern, tbc, array, clover) for the C solvers: 0 = Brillouin link array, 1 = Wilson gauge
    field; clover None or (V, 12, 12)."""
    if isinstance(W, WilsonKernel):
        return 1, W.tbc, W.U, W.clover
    if isinstance(W, BrillouinKernel):
        return 0, 0, W.W, W.clover
    return 0, 0, _c128(W), None


def clover_field(L, U: np.ndarray, csw: float) -> np.ndarray:
    """-(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu per site, (V, 12, 12), index 3*spin + colour,
    with the clover-leaf F_mu_nu (see oracle.c)."""
    V = volume(L)
    U = _c128(U)
    assert U.shape == (4, V, 3, 3)
    out = np.zeros((V, 12, 12), dtype=np.complex128)
    _load().orc_clover(_ptr(_geom(L)), _ptr(U), float(csw), _ptr(out))
    return out


def _apply(fn, L, W, m0, psi, wfn=None, adj=False):
    V = volume(L)
    psi = _c128(psi)
    squeeze = psi.ndim == 3
    if squeeze:
        psi = psi[None]
    assert psi.shape[1:] == (V, 4, 3)
    out = np.zeros_like(psi)
    kern, tbc, arr, clov = _kernel_args(W)
    if kern == 1:
        assert arr.shape == (4, V, 3, 3)
        wfn(_ptr(_geom(L)), tbc, _ptr(arr), float(m0), _ptr(psi), _ptr(out), int(psi.shape[0]))
    else:
        fn(_ptr(_geom(L)), _ptr(arr), float(m0), _ptr(psi), _ptr(out), int(psi.shape[0]))
    if clov is not None:
        _load().orc_clover_apply(_ptr(_geom(L)), _ptr(clov), _ptr(psi), _ptr(out), int(psi.shape[0]),
                                 1 if adj else 0)
    return out[0] if squeeze else out


def dirac(L, W, m0: float, psi: np.ndarray) -> np.ndarray:
    """D_bri(m0) psi, direct 81-term sum (D_wil(m0) psi for a WilsonKernel)."""
    return _apply(_load().orc_dirac, L, W, m0, psi, _load().orc_wilson)


def dirac_adj(L, W, m0: float, psi: np.ndarray) -> np.ndarray:
    """D(m0)^dag psi by the transposed sum (no gamma5 trick); Brillouin or Wilson."""
    return _apply(_load().orc_dirac_adj, L, W, m0, psi, _load().orc_wilson_adj, adj=True)


def dense_matrix(L, W, m0: float) -> np.ndarray:
    """Dense D_bri(m0) (or D_wil(m0) for a WilsonKernel), index 12*site + 3*spin + colour."""
    V = volume(L)
    n = 12 * V
    M = np.zeros((n, n), dtype=np.complex128)
    kern, tbc, arr, clov = _kernel_args(W)
    if kern == 1:
        _load().orc_wilson_dense(_ptr(_geom(L)), tbc, _ptr(arr), float(m0), _ptr(M))
    else:
        _load().orc_dirac_dense(_ptr(_geom(L)), _ptr(arr), float(m0), _ptr(M))
    if clov is not None:
        for x in range(V):
            M[12 * x:12 * x + 12, 12 * x:12 * x + 12] += clov[x]
    return M


def _apply_at(fn, L, U, tbc, m0, psi, sites):
    V = volume(L)
    U = _c128(U)
    assert U.shape == (4, V, 3, 3)
    psi = _c128(psi)
    assert psi.shape == (V, 4, 3)
    st = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((len(st), 4, 3), dtype=np.complex128)
    fn(_ptr(_geom(L)), int(tbc), _ptr(U), float(m0), _ptr(psi), len(st), _ptr(st), _ptr(out))
    return out


def dirac_at(L, U, tbc, m0: float, psi: np.ndarray, sites) -> np.ndarray:
    """(D_bri(m0) psi)(x) for x in sites, shape (len(sites), 4, 3); links from U on the fly."""
    return _apply_at(_load().orc_dirac_at, L, U, tbc, m0, psi, sites)


def dirac_adj_at(L, U, tbc, m0: float, psi: np.ndarray, sites) -> np.ndarray:
    """(D_bri(m0)^dag psi)(x) for x in sites (transposed sum, links on the fly)."""
    return _apply_at(_load().orc_dirac_adj_at, L, U, tbc, m0, psi, sites)


# -------------------------------------------------------------------- solvers


def cg(L, W, m0: float, sigma: float, b: np.ndarray, tol: float = 1e-13, maxit: int = 10000):
    """x = (D^dag D + sigma)^{-1} b by textbook CG; returns (x, iters, true_rel_resid)."""
    b = _c128(b)
    x = np.zeros_like(b)
    rel = ctypes.c_double(0)
    kern, tbc, arr, clov = _kernel_args(W)
    it = _load().orc_cg(
        _ptr(_geom(L)), kern, tbc, _ptr(arr), None if clov is None else _ptr(clov), float(m0), float(sigma), _ptr(b), _ptr(x), float(tol), int(maxit),
        ctypes.byref(rel),
    )
    return x, it, rel.value


def kl_coeffs(n: int, kind: str = "diag"):
    """(c0, omega, sigma) in double precision: g_{2n+1} (kind "diag") or g_{2n} (kind "upper",
    c0 = 0)."""
    if kind == "diag":
        return kl.kl_diag_coeffs_f64(n)
    if kind == "upper":
        om, sg = kl.kl_upper_coeffs(n)
        return 0.0, [float(v) for v in om], [float(v) for v in sg]
    raise ValueError(kind)


def rational_apply(L, W, m0: float, n: int, b: np.ndarray, tol: float = 1e-13, maxit: int = 10000,
                   kind: str = "diag", relax=False):
    """y = r_n(D^dag D) b = c0 b + sum_i omega_i (D^dag D + sigma_i)^{-1} b, shifts solved one by one.

    kind "diag": the coefficients of g_{2n+1} (eq. (KLnn_parfrac)); "upper": those of g_{2n}
    (Sec. 3.3), c0 = 0.  relax True: shift i is solved to tol * max(omega) / omega_i instead of
    tol (App. B).  relax "bound": tol bounds the error of D r_n(D^dag D) b instead, through
    |D (D^dag D + sigma)^{-1}| <= 1 / (2 sqrt(sigma)): shift i is solved to
    tol 2 sqrt(sigma_i) / (n omega_i), so that sum_i omega_i |r_i| / (2 sqrt(sigma_i)) <= tol |b|.
    Returns (y, iters per shift, true relative residual per shift)."""
    c0, om, sg = kl_coeffs(n, kind)
    if relax:
        if relax == "bound":
            tols = [tol * 2.0 * np.sqrt(s) / (n * o) for o, s in zip(om, sg)]
        else:
            wmax = max(om)
            tols = [tol * wmax / o for o in om]
        y = c0 * _c128(b)
        iters = np.zeros(n, dtype=np.int32)
        rel = np.zeros(n, dtype=np.float64)
        for i in range(n):
            yi, it_i, rel_i = rational_apply_coeffs(L, W, m0, 0.0, [om[i]], [sg[i]], b, tols[i], maxit)
            y = y + yi
            iters[i], rel[i] = it_i[0], rel_i[0]
        return y, iters, rel
    return rational_apply_coeffs(L, W, m0, c0, om, sg, b, tol, maxit)


def rational_apply_coeffs(L, W, m0: float, c0: float, om, sg, b: np.ndarray, tol: float, maxit: int):
    """y = c0 b + sum_i om_i (D^dag D + sg_i)^{-1} b for given coefficients, each shift by its own CG."""
    n = len(om)
    b = _c128(b)
    y = np.zeros_like(b)
    om = np.ascontiguousarray(om, dtype=np.float64)
    sg = np.ascontiguousarray(sg, dtype=np.float64)
    iters = np.zeros(n, dtype=np.int32)
    rel = np.zeros(n, dtype=np.float64)
    kern, tbc, arr, clov = _kernel_args(W)
    _load().orc_rational(
        _ptr(_geom(L)), kern, tbc, _ptr(arr), None if clov is None else _ptr(clov), float(m0), int(n), float(c0), _ptr(om), _ptr(sg), _ptr(b), _ptr(y),
        float(tol), int(maxit), _ptr(iters), _ptr(rel),
    )
    return y, iters, rel


def sign_apply(L, W, rho: float, n: int, b: np.ndarray, tol: float = 1e-13, maxit: int = 10000,
               kind: str = "diag", relax=False):
    """g_{2n+1}(H) b (or g_{2n}(H) b for kind "upper") with H = gamma5 D(-rho):
    g(H) = H r_n(H^2), H^2 = D^dag D, so g(H) b = gamma5 D r_n(D^dag D) b."""
    y, iters, rel = rational_apply(L, W, -rho, n, b, tol, maxit, kind, relax)
    return gamma5_apply(dirac(L, W, -rho, y)), iters, rel


def ov_apply(L, W, rho: float, n: int, b: np.ndarray, tol: float = 1e-13, maxit: int = 10000,
             kind: str = "diag", relax=False):
    """D_ov b = rho (1 + gamma5 g(H)) b = rho (b + D(-rho) r_n(D^dag D) b), eq. (def_over), with
    g = g_{2n+1} (kind "diag") or g_{2n} (kind "upper")."""
    y, iters, rel = rational_apply(L, W, -rho, n, b, tol, maxit, kind, relax)
    return rho * (b + dirac(L, W, -rho, y)), iters, rel


# ----------------------------------------------------------------- link force


def gell_mann(a: int) -> np.ndarray:
    """lambda_{a+1} (a = 0..7) as the oracle writes it out."""
    out = np.zeros(9, dtype=np.complex128)
    _load().orc_lambda(int(a), _ptr(out))
    return out.reshape(3, 3)


def link_force(L, U: np.ndarray, tbc: int, pairs, kernel: str = "bri") -> np.ndarray:
    """F (4, V, 8): dS/d omega^a_mu(z) at omega = 0 for U_mu(z) -> exp(i omega lambda_a / 2) U_mu(z),
    S = Re sum_p w_p u_p^dag D v_p with D = D_bri (kernel "bri", product rule along every path of
    every off-axis link) or D = D_wil (kernel "wil", the two hops each link enters);
    pairs = [(w, u, v), ...] with u, v of shape (V, 4, 3)."""
    V = volume(L)
    U = _c128(U)
    assert U.shape == (4, V, 3, 3)
    w = np.ascontiguousarray([float(p[0]) for p in pairs], dtype=np.float64)
    u = _c128(np.stack([np.asarray(p[1]).reshape(V, 4, 3) for p in pairs]))
    v = _c128(np.stack([np.asarray(p[2]).reshape(V, 4, 3) for p in pairs]))
    F = np.zeros((4, V, 8), dtype=np.float64)
    fn = {"bri": _load().orc_link_force, "wil": _load().orc_wilson_force}[kernel]
    fn(_ptr(_geom(L)), int(tbc), _ptr(U), len(pairs), _ptr(w), _ptr(u), _ptr(v), _ptr(F))
    return F


def ov_force(L, U: np.ndarray, tbc: int, rho: float, n: int, chi: np.ndarray, psi: np.ndarray,
             tol: float = 1e-13, maxit: int = 10000, kind: str = "diag", kernel: str = "bri"):
    """Gradient of S = Re chi^dag D_ov psi, D_ov = rho (1 + X r_n(X^dag X)), X = D_bri(-rho)
    (kernel "bri") or X = D_wil(-rho) (kernel "wil").

    With a_i = (A + sigma_i)^{-1} psi, b_i = (A + sigma_i)^{-1} X^dag chi, A = X^dag X and
    y = c0 psi + sum_i omega_i a_i, the derivative of the partial fractions gives
      dS = rho Re[chi^dag dX y] - rho sum_i omega_i Re[(X a_i)^dag dX b_i + (X b_i)^dag dX a_i],
    and grad_psi S = D_ov^dag chi = rho (chi + c0 X^dag chi + sum_i omega_i b_i).
    kind selects g_{2n+1} or g_{2n} as in rational_apply.
    Returns (F (4, V, 8), grad_psi (V, 4, 3))."""
    c0, om, sg = kl_coeffs(n, kind)
    W = links(L, U, tbc) if kernel == "bri" else WilsonKernel(U, tbc)
    m0 = -rho
    xdc = dirac_adj(L, W, m0, chi)
    pairs = []
    y = c0 * _c128(psi)
    gpsi = _c128(chi) + c0 * xdc
    for i in range(n):
        a, _, _ = cg(L, W, m0, sg[i], psi, tol, maxit)
        b, _, _ = cg(L, W, m0, sg[i], xdc, tol, maxit)
        y = y + om[i] * a
        gpsi = gpsi + om[i] * b
        pairs.append((-rho * om[i], dirac(L, W, m0, a), b))
        pairs.append((-rho * om[i], dirac(L, W, m0, b), a))
    pairs.insert(0, (rho, chi, y))
    return link_force(L, U, tbc, pairs, kernel), rho * gpsi
