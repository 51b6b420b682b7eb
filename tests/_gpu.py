"""Shared helpers of the GPU tests: seeded fields on both sides."""

import functools

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=None)
def field(L, kind, tbc=0):
    """(U numpy, oracle W) for a named link recipe."""
    L = tuple(L)
    if kind == "unit":
        U = synth.unit_links(L)
    elif kind == "rough":
        U = synth.random_links(L, 0.8, synth.LINK_SEED_BASE + 100)
    elif kind == "cfg1":
        U = synth.random_links(L, 0.3, synth.LINK_SEED_BASE + 1)
    elif kind == "cfg2":
        U = synth.smeared_links(L, 0.5, synth.LINK_SEED_BASE + 2, 0.6, 3)
    else:
        raise ValueError(kind)
    return U, oracle.links(L, U, tbc=tbc)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def round_bf16(x32: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def round_links(W: np.ndarray, prec: int) -> np.ndarray:
    """The oracle's FP64 links rounded as the library stores them (via float32)."""
    if prec == 0:
        return W
    w32 = W.astype(np.complex64)
    if prec == 1:
        return w32.astype(np.complex128)
    re = round_bf16(w32.real.copy())
    im = round_bf16(w32.imag.copy())
    return re.astype(np.float64) + 1j * im.astype(np.float64)
