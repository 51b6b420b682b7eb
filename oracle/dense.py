"""Dense small-lattice tools of the oracle (TEST INFRASTRUCTURE ONLY).

On a 4^4 lattice the Brillouin operator is a 3072 x 3072 matrix, small enough
to diagonalise.  With H = gamma5 D(-rho) Hermitian (D is gamma5-hermitian,
Sec. 4), H = Q diag(lam) Q^dag gives
  * the exact sign function  sign(H) = Q sgn(lam) Q^dag,
  * the Kenney-Laub rational g_{2n+1}(H) = Q g_{2n+1}(lam) Q^dag (same rational
    function as the multi-shift path, no Krylov solver involved),
  * the overlap operator rho (1 + gamma5 g(H)), eq. (def_over).
"""

from __future__ import annotations

import numpy as np

from . import gamma, kl


def gamma5_big(V: int) -> np.ndarray:
    g5 = gamma(4)
    return np.kron(np.eye(V), np.kron(g5, np.eye(3)))


class DenseOverlap:
    """Eigendecomposition of H = gamma5 D(-rho) for one small gauge field."""

    def __init__(self, D_kernel: np.ndarray, V: int, rho: float):
        self.V = V
        self.rho = rho
        self.D = D_kernel
        self.G5 = np.diag(gamma5_big(V)).real.copy()  # gamma5 is diagonal in the chiral basis
        H = self.G5[:, None] * D_kernel
        H = 0.5 * (H + H.conj().T)
        self.lam, self.Q = np.linalg.eigh(H)

    def fn_of_H(self, f) -> np.ndarray:
        return (self.Q * f(self.lam)[None, :]) @ self.Q.conj().T

    def apply_fn(self, f, v: np.ndarray) -> np.ndarray:
        c = self.Q.conj().T @ v
        return self.Q @ (f(self.lam) * c)

    def sign_exact_apply(self, v):
        return self.apply_fn(np.sign, v)

    def g_apply(self, n: int, v):
        return self.apply_fn(lambda lam: lam * kl.r_diag_f64(lam * lam, n), v)

    def ov_apply(self, n: int, v):
        return self.rho * (v + self.G5 * self.g_apply(n, v))

    def sign_bound(self, n: int) -> float:
        """max over the spectrum of |g_{2n+1}(lam) - sgn(lam)|."""
        lam = self.lam
        return float(np.max(np.abs(lam * kl.r_diag_f64(lam * lam, n) - np.sign(lam))))
