"""MI355X library for the Brillouin-kernel overlap operator (arXiv:1701.00726).

Thin ctypes binding of `libbrillouin.so` (the C ABI declared in
include/brillouin.h).  Every step of the computation runs in the library's HIP
kernels; this module only checks shapes, passes device pointers and the
current HIP stream, and converts between the natural (site-major) layout of
`synth` and the library's structure-of-arrays layout.

torch tensors provide device memory:
  U    complex128, shape (4, 3, 3, V)
  W    (40, 3, 3, V): complex128 (BRI_F64), complex64 (BRI_F32),
       int32 holding (re, im) bfloat16 pairs (BRI_F32_BF16W)
  psi  (nrhs, 4, 3, V): complex128 (BRI_F64) or complex64 (BRI_F32*)
  F    float64, shape (4, 8, V): link force, dS/d omega^a for
       U -> exp(i omega^a lambda_a / 2) U
  GU   complex128, shape (4, 3, 3, V): dS/dRe U + i dS/dIm U
"""

from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BRI_LIB selects another build of the library (the CPU sanitizer job's instrumented copy)
LIB_PATH = os.environ.get("BRI_LIB") or os.path.join(_HERE, "libbrillouin.so")

F64, F32, F32_BF16W = 0, 1, 2
KL_DIAG, KL_UPPER = 0, 1
RELAX_OFF, RELAX_OMEGA, RELAX_BOUND = 0, 1, 2
KERNEL_BRILLOUIN, KERNEL_WILSON = 0, 1
OK, EINVAL, ENOCONV, ENAN, EHIP, ESCRATCH = 0, -1, -2, -3, -4, -5
MAX_SHIFTS = 32
STATUS_NAMES = {OK: "BRI_OK", EINVAL: "BRI_EINVAL", ENOCONV: "BRI_ENOCONV", ENAN: "BRI_ENAN", EHIP: "BRI_EHIP",
                ESCRATCH: "BRI_ESCRATCH"}


class BriError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} returned {STATUS_NAMES.get(status, status)}")
        self.status = status


class _Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("tbc", ctypes.c_int32), ("csw", ctypes.c_double)]


class _OvParams(ctypes.Structure):
    _fields_ = [
        ("kl_n", ctypes.c_int),
        ("rho", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("inner", ctypes.c_int),
        ("max_refine", ctypes.c_int),
        ("kind", ctypes.c_int),
        ("relax", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("recompute", ctypes.c_int),
    ]


class _OvStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("refine", ctypes.c_int),
        ("shift_iters", ctypes.c_int * MAX_SHIFTS),
        ("rel_resid", ctypes.c_double * MAX_SHIFTS),
        ("seconds", ctypes.c_double),
    ]


class _MassParams(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double),
        ("complete", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
    ]


MAX_LEVELS = 4
MAX_SOLVE_RHS = 16


class _Level(ctypes.Structure):
    _fields_ = [
        ("kl_n", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("ms_tol", ctypes.c_double),
        ("inner", ctypes.c_int),
    ]


class _SolveStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("inner_iters", ctypes.c_int),
        ("applies", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("level_iters", ctypes.c_int * MAX_LEVELS),
        ("level_calls", ctypes.c_int * MAX_LEVELS),
        ("level_applies", ctypes.c_int * MAX_LEVELS),
        ("seconds", ctypes.c_double),
    ]


class StencilCfg(ctypes.Structure):
    """Launch configuration of the stencil kernels (see include/brillouin.h)."""

    _fields_ = [
        ("tile_x", ctypes.c_int),
        ("tile_y", ctypes.c_int),
        ("tile_z", ctypes.c_int),
        ("tile_t", ctypes.c_int),
        ("col_z", ctypes.c_int),
        ("nsplit", ctypes.c_int),
        ("rpt", ctypes.c_int),
        ("xcd", ctypes.c_int),
        ("variant", ctypes.c_int),
        ("col_y", ctypes.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


@dataclass
class OvStats:
    iters: int
    refine: int
    shift_iters: list = field(default_factory=list)
    rel_resid: list = field(default_factory=list)
    seconds: float = 0.0


@dataclass
class SolveStats:
    iters: int
    inner_iters: int
    applies: int
    rel_resid: float
    seconds: float = 0.0
    level_iters: list = field(default_factory=list)
    level_calls: list = field(default_factory=list)
    level_applies: list = field(default_factory=list)


@dataclass
class Level:
    """One preconditioner level of the cascaded solve (Sec. 8): kl_n = 0 is the Brillouin
    operator rho D_bri(-rho) + rho + mt (last level only), kl_n > 0 the overlap approximant of
    that Kenney-Laub order plus mt.  It is inverted by BiCGstab to `tol` (relative) or
    `max_iter` iterations; its multi-shift runs at `ms_tol` in precision `inner`."""
    kl_n: int
    tol: float = 0.1
    max_iter: int = 50
    ms_tol: float = 1e-4
    inner: int = 0


_lock = threading.Lock()
_lib = None


def load():
    """Load libbrillouin.so; raises if it was not built (no fallback path exists)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with `python -m paper_1701_00726_amd.build` "
                    "(the library has no CPU fallback)"
                )
            lib = ctypes.CDLL(LIB_PATH)
            P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
            G = ctypes.POINTER(_Geom)
            lib.bri_build_links.argtypes = [G, P, P, I, P]
            lib.bri_round_links.argtypes = [G, P, P, I, P]
            lib.bri_apply.argtypes = [G, P, I, D, P, P, I, P]
            lib.bri_apply_dag.argtypes = [G, P, I, D, P, P, I, P]
            lib.wil_apply.argtypes = [G, P, I, D, P, P, I, P]
            lib.wil_apply_dag.argtypes = [G, P, I, D, P, P, I, P]
            ovargs = [G, P, P, ctypes.POINTER(_OvParams), P, P, I, P, ctypes.POINTER(ctypes.c_size_t),
                      ctypes.POINTER(_OvStats), P]
            lib.ov_sign_apply.argtypes = ovargs
            lib.ov_apply.argtypes = ovargs
            lib.ov_apply_noalloc.argtypes = [G, P, P, ctypes.POINTER(_OvParams), P, P, I, ctypes.POINTER(_OvStats), P]
            lib.ov_noalloc_max_bytes.argtypes = []
            lib.bri_kl_coeffs.argtypes = [I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
            SC = ctypes.POINTER(StencilCfg)
            lib.bri_stencil_time.argtypes = [G, P, I, P, P, I, SC, I, ctypes.POINTER(D), P]
            lib.bri_autotune.argtypes = [G, P, I, P, P, I, I, SC, ctypes.POINTER(D), P]
            lib.bri_set_stencil_cfg.argtypes = [G, I, I, SC]
            lib.bri_get_stencil_cfg.argtypes = [G, I, I, SC]
            lib.bri_set_solver_graphs.argtypes = [I]
            SZ = ctypes.POINTER(ctypes.c_size_t)
            lib.bri_link_grad.argtypes = [G, P, P, I, ctypes.POINTER(D), P, P, P, P, P, SZ, P]
            lib.wil_link_grad.argtypes = [G, P, P, I, ctypes.POINTER(D), P, P, P, P, P, SZ, P]
            lib.bri_kl_upper_coeffs.argtypes = [I, ctypes.POINTER(D), ctypes.POINTER(D)]
            lib.ov_solve.argtypes = [G, P, P, ctypes.POINTER(_OvParams), ctypes.POINTER(_MassParams), I,
                                     ctypes.POINTER(_Level), P, P, I, P, SZ, ctypes.POINTER(_SolveStats), P]
            lib.ov_apply_grad.argtypes = [G, P, P, P, ctypes.POINTER(_OvParams), P, P, P, P, P, P, SZ,
                                          ctypes.POINTER(_OvStats), P]
            for fn in EXPORTS:
                getattr(lib, fn).restype = I
            lib.ov_noalloc_max_bytes.restype = ctypes.c_size_t
            _lib = lib
    return _lib


EXPORTS = (
    "bri_build_links",
    "bri_round_links",
    "bri_apply",
    "bri_apply_dag",
    "wil_apply",
    "wil_apply_dag",
    "ov_sign_apply",
    "ov_apply",
    "bri_kl_coeffs",
    "bri_stencil_time",
    "bri_autotune",
    "bri_set_stencil_cfg",
    "bri_get_stencil_cfg",
    "bri_link_grad",
    "wil_link_grad",
    "ov_apply_grad",
    "ov_solve",
    "bri_kl_upper_coeffs",
    "bri_set_solver_graphs",
    "ov_apply_noalloc",
    "ov_noalloc_max_bytes",
)
MAX_PAIRS = 2 * MAX_SHIFTS + 1


# ------------------------------------------------------------------ helpers


def _torch():
    import torch

    return torch


def _geom(L, tbc=0, csw=0.0):
    g = _Geom()
    for i in range(4):
        g.L[i] = int(L[i])
    g.tbc = int(tbc)
    g.csw = float(csw)
    return g


def _clover_flag(W):
    """csw for the geometry of an apply: the applies read the clover field from the link array
    (48 slabs: 40 link slabs and 8 of clover entries) and only test csw != 0."""
    return 1.0 if W.shape[0] == 48 else 0.0


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check_out(out, dtype, shape, device):
    """A caller-supplied output must be exactly what the kernels write: dtype, shape, device."""
    if out.dtype != dtype or tuple(out.shape) != tuple(shape) or out.device != device:
        raise ValueError(f"out must be {dtype} of shape {tuple(shape)} on {device}")
    return out


def _check(fn, status, allow=()):
    if status != OK and status not in allow:
        raise BriError(fn, status)
    return status


def spinor_dtype(prec):
    torch = _torch()
    return torch.complex128 if prec == F64 else torch.complex64


def link_dtype(prec):
    torch = _torch()
    return {F64: torch.complex128, F32: torch.complex64, F32_BF16W: torch.int32}[prec]


# ------------------------------------------------------------ layout helpers


def links_to_device(U_np, device="cuda"):
    """(4, V, 3, 3) complex128 numpy -> (4, 3, 3, V) device tensor."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(np.transpose(U_np, (0, 2, 3, 1)))).to(device)


def spinor_to_device(psi_np, prec=F64, device="cuda"):
    """(nrhs, V, 4, 3) numpy -> (nrhs, 4, 3, V) device tensor."""
    torch = _torch()
    a = np.ascontiguousarray(np.transpose(psi_np, (0, 2, 3, 1)))
    return torch.from_numpy(a).to(device=device, dtype=spinor_dtype(prec))


def spinor_to_host(psi_t):
    """(nrhs, 4, 3, V) tensor -> (nrhs, V, 4, 3) complex128 numpy."""
    a = psi_t.detach().to("cpu").numpy().astype(np.complex128)
    return np.ascontiguousarray(np.transpose(a, (0, 3, 1, 2)))


def clover_to_host(W_t, prec=F64):
    """The clover term stored after the link slabs of a (48, 3, 3, V) array, as (V, 12, 12)
    complex128 (block diagonal in the two chiralities)."""
    V = W_t.shape[-1]
    a = links_W_to_host(W_t, prec)[:, 40:].reshape(V, 2, 6, 6)
    out = np.zeros((V, 12, 12), dtype=np.complex128)
    out[:, :6, :6] = a[:, 0]
    out[:, 6:, 6:] = a[:, 1]
    return out


def links_W_to_host(W_t, prec=F64):
    """(40, 3, 3, V) tensor -> (V, 40, 3, 3) complex128 numpy (bfloat16 pairs unpacked)."""
    if prec == F32_BF16W:
        u = W_t.detach().to("cpu").numpy().view(np.uint32)
        re = ((u & 0xFFFF).astype(np.uint32) << 16).view(np.float32)
        im = (u & 0xFFFF0000).astype(np.uint32).view(np.float32)
        a = re.astype(np.complex128) + 1j * im.astype(np.float64)
    else:
        a = W_t.detach().to("cpu").numpy().astype(np.complex128)
    return np.ascontiguousarray(np.transpose(a, (3, 0, 1, 2)))


# ------------------------------------------------------------------ the ABI


def build_links(L, U, prec=F64, tbc=0, stream=None, out=None, csw=0.0):
    """Off-axis links W [40][3][3][V] in precision `prec` from device links U [4][3][3][V];
    with csw != 0 the clover term follows as 8 more slabs ([48][3][3][V] in all, the clover
    entries [2][6][6][V] after the links)."""
    torch = _torch()
    V = int(np.prod(L))
    if U.dtype != torch.complex128 or tuple(U.shape) != (4, 3, 3, V):
        raise ValueError("U must be complex128 of shape (4, 3, 3, V)")
    nslab = 48 if csw else 40
    if out is None:
        out = torch.empty((nslab, 3, 3, V), dtype=link_dtype(prec), device=U.device)
    _check_out(out, link_dtype(prec), (nslab, 3, 3, V), U.device)
    g = _geom(L, tbc, csw)
    _check("bri_build_links", load().bri_build_links(ctypes.byref(g), _dptr(U), _dptr(out), int(prec), _stream(stream)))
    return out


def round_links(L, W64, prec, stream=None, out=None):
    """The FP64 link array W64 of build_links rounded to prec (F32 or F32_BF16W), as build_links
    would store it; no allocation in the library."""
    torch = _torch()
    V = int(np.prod(L))
    if W64.dtype != torch.complex128 or W64.shape[0] not in (40, 48) or tuple(W64.shape[1:]) != (3, 3, V):
        raise ValueError("W64 must be complex128 of shape (40 or 48, 3, 3, V)")
    if out is None:
        out = torch.empty(tuple(W64.shape), dtype=link_dtype(prec), device=W64.device)
    _check_out(out, link_dtype(prec), tuple(W64.shape), W64.device)
    g = _geom(L, 0, _clover_flag(W64))
    _check("bri_round_links", load().bri_round_links(ctypes.byref(g), _dptr(W64), _dptr(out), int(prec),
                                                     _stream(stream)))
    return out


def _apply(fn, L, W, prec, m0, psi, out=None, stream=None):
    torch = _torch()
    V = int(np.prod(L))
    if psi.dim() != 4 or tuple(psi.shape[1:]) != (4, 3, V) or psi.dtype != spinor_dtype(prec):
        raise ValueError("psi must be (nrhs, 4, 3, V) of the spinor dtype of prec")
    if W.dtype != link_dtype(prec) or W.shape[0] not in (40, 48) or tuple(W.shape[1:]) != (3, 3, V):
        raise ValueError("W must be (40 or 48, 3, 3, V) of the link dtype of prec")
    if out is None:
        out = torch.empty_like(psi)
    _check_out(out, psi.dtype, psi.shape, psi.device)
    g = _geom(L, 0, _clover_flag(W))
    st = getattr(load(), fn)(ctypes.byref(g), _dptr(W), int(prec), float(m0), _dptr(psi), _dptr(out),
                             int(psi.shape[0]), _stream(stream))
    _check(fn, st)
    return out


def apply(L, W, prec, m0, psi, out=None, stream=None):
    """out = D_bri(m0) psi."""
    return _apply("bri_apply", L, W, prec, m0, psi, out, stream)


def apply_dag(L, W, prec, m0, psi, out=None, stream=None):
    """out = D_bri(m0)^dag psi."""
    return _apply("bri_apply_dag", L, W, prec, m0, psi, out, stream)


def wilson_apply(L, W, prec, m0, psi, out=None, stream=None):
    """out = D_wil(m0) psi, reading the one-hop slabs of the link array W."""
    return _apply("wil_apply", L, W, prec, m0, psi, out, stream)


def wilson_apply_dag(L, W, prec, m0, psi, out=None, stream=None):
    """out = D_wil(m0)^dag psi."""
    return _apply("wil_apply_dag", L, W, prec, m0, psi, out, stream)


class OverlapOp:
    """Holds the workspace of ov_apply / ov_sign_apply for one lattice and parameter set."""

    def __init__(self, L, W64, kl_n=16, rho=1.0, tol=1e-12, max_iter=2000, Wlo=None, inner=F64, tbc=0,
                 max_refine=None, nrhs=1, kind=KL_DIAG, relax=False, kernel=KERNEL_BRILLOUIN, recompute=0):
        """Workspace for up to `nrhs` right-hand sides per call.  inner = F32 or
        F32_BF16W runs the late multi-shift iterations (once the residual has fallen to
        tol / unit roundoff) on FP32 vectors with the low-precision links `Wlo`,
        accumulating the result in FP64 (max_refine is unused).  kind = KL_UPPER
        uses the first upper diagonal g_{2n} instead of g_{2n+1}; relax = RELAX_OMEGA (or True)
        stops shift i at tol * omega_max / omega_i, RELAX_BOUND stops once the bound
        sum_i omega_i |r_i| / (2 sqrt(sigma_i)) on the error of sign(H) psi is at most
        tol |psi|; kernel = KERNEL_WILSON builds the overlap on the
        Wilson operator (the one-hop slabs of W64) instead of the Brillouin one.  recompute = m > 0
        makes grad solve the shifts m at a time, keeping only those solutions (less memory,
        more solver iterations); 0 keeps all of one multi-shift solve."""
        self.L = tuple(int(v) for v in L)
        if Wlo is not None and Wlo.shape[0] != W64.shape[0]:
            raise ValueError("W64 and Wlo must both carry the clover term or both not")
        self.g = _geom(self.L, tbc, _clover_flag(W64))
        self.W64 = W64
        self.Wlo = Wlo
        if inner != F64 and Wlo is None:
            raise ValueError("a low-precision inner solve needs Wlo")
        if max_refine is None:
            max_refine = 0
        self.params = _OvParams(int(kl_n), float(rho), float(tol), int(max_iter), int(inner), int(max_refine),
                                int(kind), int(relax), int(kernel), int(recompute))
        self.nrhs = int(nrhs)
        nbytes = ctypes.c_size_t(0)
        _check(
            "ov_apply",
            load().ov_apply(ctypes.byref(self.g), None, None, ctypes.byref(self.params), None, None, self.nrhs, None,
                            ctypes.byref(nbytes), None, None),
        )
        torch = _torch()
        self.work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=W64.device)
        self.work_bytes = nbytes.value

    def _run(self, fn, psi, out, stream, allow_noconv):
        torch = _torch()
        V = int(np.prod(self.L))
        if psi.dtype != torch.complex128 or psi.dim() != 4 or tuple(psi.shape[1:]) != (4, 3, V):
            raise ValueError("psi must be complex128 (nrhs, 4, 3, V)")
        if psi.shape[0] > self.nrhs:
            raise ValueError(f"workspace sized for {self.nrhs} right-hand sides, got {psi.shape[0]}")
        if out is None:
            out = torch.empty_like(psi)
        _check_out(out, psi.dtype, psi.shape, psi.device)
        stats = _OvStats()
        wb = ctypes.c_size_t(self.work_bytes)
        st = getattr(load(), fn)(
            ctypes.byref(self.g), _dptr(self.W64), None if self.Wlo is None else _dptr(self.Wlo),
            ctypes.byref(self.params), _dptr(psi), _dptr(out), int(psi.shape[0]), _dptr(self.work), ctypes.byref(wb),
            ctypes.byref(stats), _stream(stream),
        )
        _check(fn, st, allow=(ENOCONV,) if allow_noconv else ())
        n = self.params.kl_n
        s = OvStats(stats.iters, stats.refine, list(stats.shift_iters[:n]), list(stats.rel_resid[:n]), stats.seconds)
        s.status = st
        return out, s

    def apply(self, psi, out=None, stream=None, allow_noconv=False):
        """out = D_ov psi = rho (psi + X r_n(X^dag X) psi)."""
        return self._run("ov_apply", psi, out, stream, allow_noconv)

    def sign(self, psi, out=None, stream=None, allow_noconv=False):
        """out = sign(H) psi ~= gamma5 X r_n(X^dag X) psi."""
        return self._run("ov_sign_apply", psi, out, stream, allow_noconv)

    def grad(self, U, chi, psi, force=True, link_grad=False, stream=None, allow_noconv=False):
        """Gradient of S = Re chi^dag D_ov psi for one right-hand side.

        U is the (4, 3, 3, V) complex128 field W64 was built from (with this
        operator's tbc).  The shift solves run in this operator's inner precision
        (low-precision late iterations as in apply).  Returns (F or None, GU or None, grad_psi, OvStats) with
        F (4, 8, V) the force, GU (4, 3, 3, V) = dS/dRe U + i dS/dIm U and
        grad_psi = D_ov^dag chi of the shape of psi."""
        torch = _torch()
        V = int(np.prod(self.L))
        for name, t in (("chi", chi), ("psi", psi)):
            if t.dtype != torch.complex128 or t.numel() != 12 * V:
                raise ValueError(f"{name} must be complex128 with 12 V elements")
        if U.dtype != torch.complex128 or tuple(U.shape) != (4, 3, 3, V):
            raise ValueError("U must be complex128 of shape (4, 3, 3, V)")
        if not (force or link_grad):
            raise ValueError("ask for the force, the link gradient or both")
        if getattr(self, "_gwork", None) is None:
            nb = ctypes.c_size_t(0)
            _check("ov_apply_grad", load().ov_apply_grad(ctypes.byref(self.g), None, None, None,
                                                         ctypes.byref(self.params), None, None, None, None, None, None,
                                                         ctypes.byref(nb), None, None))
            self._gwork = torch.empty(int(nb.value), dtype=torch.uint8, device=self.W64.device)
        F = torch.empty((4, 8, V), dtype=torch.float64, device=U.device) if force else None
        GU = torch.empty_like(U) if link_grad else None
        gpsi = torch.empty_like(psi)
        stats = _OvStats()
        wb = ctypes.c_size_t(self._gwork.numel())
        st = load().ov_apply_grad(
            ctypes.byref(self.g), _dptr(U), _dptr(self.W64), None if self.Wlo is None else _dptr(self.Wlo),
            ctypes.byref(self.params), _dptr(chi), _dptr(psi),
            None if F is None else _dptr(F), None if GU is None else _dptr(GU), _dptr(gpsi), _dptr(self._gwork),
            ctypes.byref(wb), ctypes.byref(stats), _stream(stream),
        )
        _check("ov_apply_grad", st, allow=(ENOCONV,) if allow_noconv else ())
        n = self.params.kl_n
        s = OvStats(stats.iters, stats.refine, list(stats.shift_iters[:n]), list(stats.rel_resid[:n]), stats.seconds)
        s.status = st
        return F, GU, gpsi, s


    def solve(self, b, mass, complete=True, tol=1e-10, max_iter=1000, prec=(), stream=None, allow_noconv=False):
        """x = (D_ov + mt)^{-1} bt for the right-hand sides b, (nrhs, 4, 3, V) or one source of
        12 V entries: the massive overlap equation of Sec. 4 (complete or traditional form),
        BiCGstab outer solver with every D_ov apply run by this operator, optionally right-
        preconditioned by the cascade `prec` (a sequence of Level, Sec. 8).  All right-hand
        sides run side by side.  Returns (x of the shape of b, SolveStats)."""
        torch = _torch()
        V = int(np.prod(self.L))
        if b.dtype != torch.complex128 or b.numel() % (12 * V) or b.numel() == 0:
            raise ValueError("b must be complex128 with a multiple of 12 V elements")
        nrhs = b.numel() // (12 * V)
        if nrhs > MAX_SOLVE_RHS:
            raise ValueError(f"at most {MAX_SOLVE_RHS} right-hand sides per solve")
        if not b.is_contiguous():
            raise ValueError("b must be contiguous")
        mp = _MassParams(float(mass), 1 if complete else 0, float(tol), int(max_iter))
        nprec = len(prec)
        lv = (_Level * max(nprec, 1))(*[_Level(int(l.kl_n), float(l.tol), int(l.max_iter), float(l.ms_tol),
                                                int(l.inner)) for l in prec])
        nb = ctypes.c_size_t(0)
        _check("ov_solve", load().ov_solve(ctypes.byref(self.g), None, None, ctypes.byref(self.params),
                                           ctypes.byref(mp), nprec, lv, None, None, nrhs, None, ctypes.byref(nb), None,
                                           None))
        if getattr(self, "_swork", None) is None or self._swork.numel() < nb.value:
            self._swork = None
            self._swork = torch.empty(int(nb.value), dtype=torch.uint8, device=self.W64.device)
        x = torch.empty_like(b)
        st = _SolveStats()
        wb = ctypes.c_size_t(self._swork.numel())
        rc = load().ov_solve(
            ctypes.byref(self.g), _dptr(self.W64), None if self.Wlo is None else _dptr(self.Wlo),
            ctypes.byref(self.params), ctypes.byref(mp), nprec, lv, _dptr(b), _dptr(x), nrhs, _dptr(self._swork),
            ctypes.byref(wb), ctypes.byref(st), _stream(stream),
        )
        _check("ov_solve", rc, allow=(ENOCONV,) if allow_noconv else ())
        s = SolveStats(st.iters, st.inner_iters, st.applies, st.rel_resid, st.seconds,
                       list(st.level_iters[:nprec]), list(st.level_calls[:nprec]), list(st.level_applies[:nprec]))
        s.status = rc
        return x, s


def set_solver_graphs(enable):
    """Turn HIP-graph replay of the multi-shift CG loop on (default) or off."""
    _check("bri_set_solver_graphs", load().bri_set_solver_graphs(1 if enable else 0))


def kl_upper_coeffs(n):
    """(omega[n], sigma[n]) of g_{2n} as computed by the library's host code."""
    om = (ctypes.c_double * n)()
    sg = (ctypes.c_double * n)()
    _check("bri_kl_upper_coeffs", load().bri_kl_upper_coeffs(int(n), om, sg))
    return list(om), list(sg)


def kl_coeffs(n):
    """(c0, omega[n], sigma[n]) as computed by the library's host code."""
    c0 = ctypes.c_double()
    om = (ctypes.c_double * n)()
    sg = (ctypes.c_double * n)()
    _check("bri_kl_coeffs", load().bri_kl_coeffs(int(n), ctypes.byref(c0), om, sg))
    return c0.value, list(om), list(sg)


# ------------------------------------------------------------------ autotuner


def _tune_check(L, W, prec, psi):
    V = int(np.prod(L))
    torch = _torch()
    if psi.dim() != 4 or tuple(psi.shape[1:]) != (4, 3, V) or psi.dtype != spinor_dtype(prec):
        raise ValueError("psi must be (nrhs, 4, 3, V) of the spinor dtype of prec")
    if W.dtype != link_dtype(prec) or W.shape[0] not in (40, 48) or tuple(W.shape[1:]) != (3, 3, V):
        raise ValueError("W must be (40 or 48, 3, 3, V) of the link dtype of prec")
    return torch.empty_like(psi)


def stencil_time(L, W, prec, psi, cfg=None, reps=10, stream=None):
    """Microseconds per bri_apply launch with configuration cfg (None: current default)."""
    out = _tune_check(L, W, prec, psi)
    us = ctypes.c_double()
    g = _geom(L, 0, _clover_flag(W))
    _check("bri_stencil_time", load().bri_stencil_time(ctypes.byref(g), _dptr(W), int(prec), _dptr(psi), _dptr(out),
                                                       int(psi.shape[0]), None if cfg is None else ctypes.byref(cfg),
                                                       int(reps), ctypes.byref(us), _stream(stream)))
    return us.value


def autotune(L, W, prec, psi, reps=5, stream=None):
    """Time the candidate stencil configurations for this lattice, precision and
    number of right-hand sides; the fastest is installed for later calls.
    Returns (StencilCfg, microseconds per launch)."""
    out = _tune_check(L, W, prec, psi)
    best = StencilCfg()
    us = ctypes.c_double()
    g = _geom(L, 0, _clover_flag(W))
    _check("bri_autotune", load().bri_autotune(ctypes.byref(g), _dptr(W), int(prec), _dptr(psi), _dptr(out),
                                               int(psi.shape[0]), int(reps), ctypes.byref(best), ctypes.byref(us),
                                               _stream(stream)))
    return best, us.value


def get_stencil_cfg(L, prec, nrhs):
    cfg = StencilCfg()
    g = _geom(L)
    _check("bri_get_stencil_cfg", load().bri_get_stencil_cfg(ctypes.byref(g), int(prec), int(nrhs), ctypes.byref(cfg)))
    return cfg


def set_stencil_cfg(L, prec, nrhs, cfg):
    """Install cfg (a StencilCfg) for (L, prec, nrhs); None removes the entry."""
    g = _geom(L)
    _check("bri_set_stencil_cfg", load().bri_set_stencil_cfg(ctypes.byref(g), int(prec), int(nrhs),
                                                             None if cfg is None else ctypes.byref(cfg)))


# -------------------------------------------------------------- differentiation


def link_grad(L, U, W, pairs, tbc=0, force=True, link_grad=False, stream=None, kernel=KERNEL_BRILLOUIN):
    """Gradient of S = Re sum_p w_p u_p^dag D v_p with respect to the links, D = D_bri (or
    D_wil for kernel = KERNEL_WILSON).

    pairs = [(w, u, v), ...] with u, v complex128 tensors of 12 V elements in the
    (4, 3, V) spinor layout; W the FP64 off-axis links built from U with `tbc`.
    Returns (F (4, 8, V) or None, GU (4, 3, 3, V) or None)."""
    torch = _torch()
    V = int(np.prod(L))
    if not 1 <= len(pairs) <= MAX_PAIRS:
        raise ValueError(f"1..{MAX_PAIRS} pairs")
    if U.dtype != torch.complex128 or tuple(U.shape) != (4, 3, 3, V):
        raise ValueError("U must be complex128 of shape (4, 3, 3, V)")
    if W.dtype != torch.complex128 or tuple(W.shape) != (40, 3, 3, V):
        raise ValueError("W must be the complex128 (40, 3, 3, V) links")
    if not (force or link_grad):
        raise ValueError("ask for the force, the link gradient or both")
    for _, u, v in pairs:
        if u.dtype != torch.complex128 or v.dtype != torch.complex128 or u.numel() != 12 * V or v.numel() != 12 * V:
            raise ValueError("u and v must be complex128 with 12 V elements")
    uu = torch.stack([p[1].reshape(4, 3, V) for p in pairs]).contiguous()
    vv = torch.stack([p[2].reshape(4, 3, V) for p in pairs]).contiguous()
    w = (ctypes.c_double * len(pairs))(*[float(p[0]) for p in pairs])
    g = _geom(L, tbc)
    nb = ctypes.c_size_t(0)
    lib = load()
    fname = "wil_link_grad" if kernel == KERNEL_WILSON else "bri_link_grad"
    fn = getattr(lib, fname)
    _check(fname, fn(ctypes.byref(g), None, None, len(pairs), w, None, None, None, None, None,
                                              ctypes.byref(nb), None))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=U.device)
    F = torch.empty((4, 8, V), dtype=torch.float64, device=U.device) if force else None
    GU = torch.empty_like(U) if link_grad else None
    _check(fname, fn(ctypes.byref(g), _dptr(U), _dptr(W), len(pairs), w, _dptr(uu),
                                              _dptr(vv), None if F is None else _dptr(F),
                                              None if GU is None else _dptr(GU), _dptr(work), ctypes.byref(nb),
                                              _stream(stream)))
    return F, GU



class BrillouinApply:
    """out = D_bri(m0)[U] psi as a torch.autograd.Function over (U, psi).

    Forward builds the FP64 off-axis links from U and applies the stencil; backward
    returns D_bri^dag grad_out for psi and dS/dRe U + i dS/dIm U (torch's complex
    convention) for U, both from the library's kernels.  psi has shape (nrhs, 4, 3, V)."""

    _fn = None

    @classmethod
    def apply(cls, U, psi, L, m0, tbc=0):
        if cls._fn is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, U, psi, L, m0, tbc):
                    W = build_links(L, U, F64, tbc)
                    out = apply(L, W, F64, m0, psi.contiguous())
                    ctx.save_for_backward(U, W, psi)
                    ctx.L, ctx.m0, ctx.tbc = L, m0, tbc
                    return out

                @staticmethod
                def backward(ctx, gout):
                    U, W, psi = ctx.saved_tensors
                    gout = gout.contiguous()
                    gU = gpsi = None
                    if ctx.needs_input_grad[1]:
                        gpsi = apply_dag(ctx.L, W, F64, ctx.m0, gout)
                    if ctx.needs_input_grad[0]:
                        pairs = [(1.0, gout[r], psi[r]) for r in range(psi.shape[0])]
                        GU = None
                        for k in range(0, len(pairs), MAX_PAIRS):
                            _, part = link_grad(ctx.L, U, W, pairs[k:k + MAX_PAIRS], ctx.tbc, force=False,
                                                link_grad=True)
                            GU = part if GU is None else GU + part
                        gU = GU
                    return gU, gpsi, None, None, None

            cls._fn = _Fn
        return cls._fn.apply(U, psi, tuple(int(v) for v in L), float(m0), int(tbc))


class OverlapApply:
    """out = D_ov[U] psi (one right-hand side, FP64) as a torch.autograd.Function.

    Forward: off-axis links from U, then ov_apply.  Backward: ov_apply_grad, which
    re-solves the shifted systems for psi and X^dag grad_out and returns
    dS/dRe U + i dS/dIm U for U and D_ov^dag grad_out for psi."""

    _fn = None

    @classmethod
    def apply(cls, U, psi, L, kl_n=16, rho=1.0, tol=1e-12, max_iter=2000, tbc=0):
        if cls._fn is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, U, psi, L, kl_n, rho, tol, max_iter, tbc):
                    W = build_links(L, U, F64, tbc)
                    op = OverlapOp(L, W, kl_n=kl_n, rho=rho, tol=tol, max_iter=max_iter, tbc=tbc)
                    out, _ = op.apply(psi.reshape(1, 4, 3, -1).contiguous())
                    ctx.save_for_backward(U, psi)
                    ctx.op = op
                    return out.reshape(psi.shape)

                @staticmethod
                def backward(ctx, gout):
                    U, psi = ctx.saved_tensors
                    _, GU, gpsi, _ = ctx.op.grad(U, gout.contiguous(), psi.contiguous(), force=False,
                                                 link_grad=True)
                    return (GU if ctx.needs_input_grad[0] else None,
                            gpsi.reshape(psi.shape) if ctx.needs_input_grad[1] else None,
                            None, None, None, None, None, None)

            cls._fn = _Fn
        return cls._fn.apply(U, psi, tuple(int(v) for v in L), int(kl_n), float(rho), float(tol), int(max_iter),
                             int(tbc))
