"""Linear solves for the oracle.

Small systems use a direct LU factorisation (numpy dense, or scipy's sparse
SuperLU); large ones use conjugate gradients on the normal equations
``A^dagger A x = A^dagger b``: a different algorithm from the GPU's flexible
GCR, so that an error in one is not mirrored by the other. ``cgne`` stops on
the true relative residual ``|b - A x| / |b|``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def norm2(a: np.ndarray) -> float:
    return float(np.vdot(a.reshape(-1), a.reshape(-1)).real)


def cgne(apply_A, apply_Adag, b: np.ndarray, tol: float = 1e-14, max_iter: int = 200000,
         x0: np.ndarray | None = None):
    """Solve ``A x = b`` by CG on ``A^dagger A x = A^dagger b``.

    Returns ``(x, iterations, true_relative_residual)``."""
    bn = np.sqrt(norm2(b))
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    x = np.zeros_like(b) if x0 is None else x0.copy()
    it = 0
    while True:
        r = b - apply_A(x)
        rel = np.sqrt(norm2(r)) / bn
        if rel <= tol or it >= max_iter:
            return x, it, rel
        # CG on the normal equations from the current x
        z = apply_Adag(r)
        p = z.copy()
        zz = norm2(z)
        for _ in range(2000):
            q = apply_A(p)
            alpha = zz / norm2(q)
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            if np.sqrt(norm2(r)) / bn <= 0.1 * tol:
                break
            z = apply_Adag(r)
            zz_new = norm2(z)
            p = z + (zz_new / zz) * p
            zz = zz_new


class DenseLU:
    """Dense LU (LAPACK getrf) of a square matrix; ``solve`` works on flat vectors."""

    def __init__(self, A: np.ndarray):
        import scipy.linalg as sla

        self._lu = sla.lu_factor(A)

    def solve(self, b: np.ndarray) -> np.ndarray:
        import scipy.linalg as sla

        return sla.lu_solve(self._lu, b.reshape(-1)).reshape(b.shape)


class SparseLU:
    """Sparse LU (SuperLU) of a square sparse matrix; ``solve`` works on flat vectors."""

    def __init__(self, A):
        self.n = A.shape[0]
        self._lu = spla.splu(A.tocsc())

    def solve(self, b: np.ndarray) -> np.ndarray:
        return self._lu.solve(b.reshape(-1)).reshape(b.shape)


def dense_logdet(A: np.ndarray) -> complex:
    """``ln det A`` (complex, principal branch of the phase) by LU."""
    sign, logabs = np.linalg.slogdet(A)
    return complex(logabs + np.log(sign))
