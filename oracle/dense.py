"""Dense quadrature of the integral operator (TEST INFRASTRUCTURE).

Imported only by tests, the smoke check and the bench's CPU baseline.

eq. (1.1): ``Hu(x) = int K(x, y) u(y) dy`` with the kernel recovered from the
TVIR of the introduction, ``K(x, y) = T(x - y, y)``.  On the grid
``y_j = j/N`` the rectangle rule gives ``K[i, j] = (1/N) T(lam(i - j), y_j)``,
where ``lam`` is the signed lag on the circle in [-1/2, 1/2).  The adjoint is
the transpose (real kernel).  This is the *approximated* operator, not the
parity target of the expansion: it measures how well ``H_m`` approximates
``H``.
"""
from __future__ import annotations

import numpy as np

__all__ = ["lag_of", "kernel_matrix_1d", "tvir_matrix_1d", "apply_dense",
           "adjoint_dense", "hs_norm"]


def lag_of(d, n):
    """Signed lag on the unit circle of the index difference ``d`` (mod n)."""
    d = np.asarray(d) % n
    return (((d + n // 2) % n) - n // 2) / n


def kernel_matrix_1d(T, n: int) -> np.ndarray:
    """``K[i, j] = (1/n) T(lam(i - j), y_j)``."""
    i = np.arange(n)
    y = i / n
    lam = lag_of(i[:, None] - i[None, :], n)
    return T(lam, np.broadcast_to(y[None, :], (n, n))) / n


def tvir_matrix_1d(T, n: int) -> np.ndarray:
    """``TT[l, j] = T(lam(l), y_j)``: row = lag, column = source position."""
    i = np.arange(n)
    lam = lag_of(i, n)
    return T(lam[:, None], np.broadcast_to((i / n)[None, :], (n, n)))


def apply_dense(K, u):
    """``(Hu)[i] = sum_j K[i, j] u[j]`` (batched over leading axes)."""
    return np.asarray(u, np.float64) @ K.T


def adjoint_dense(K, v):
    """``(H^* v)[j] = sum_i K[i, j] v[i]``."""
    return np.asarray(v, np.float64) @ K


def hs_norm(K) -> float:
    """Discrete Hilbert-Schmidt (Frobenius) norm; by section 3.1 it equals the
    L2 norm of the TVIR."""
    return float(np.sqrt(np.sum(np.asarray(K, np.float64) ** 2)))
