"""Constructions of ``(w_k, h_k)`` from a TVIR (TEST INFRASTRUCTURE).

Imported only by tests.  The GPU library takes ``w_k`` and ``h_k`` as given;
these routines exist to reproduce the approximation-rate statements.

* ``project``: section 4.2's B-spline projection.  For every lag ``x`` the
  coefficients ``c_k(x)`` minimise ``||T(x, .) - sum_k c_k w_k||_2`` over the
  grid; then ``h_k = c_k / N`` (rectangle-rule weight) and ``T_m(x, y) =
  sum_k c_k(x) w_k(y)`` (eq. 3.8, the low-rank TVIR of the expansion).
* ``interpolate``: section 4.4.  ``c_k(x)`` solves
  ``sum_k c_k(x) w_k(y_i) = T(x, y_i)`` at the ``m`` nodes ``y_i``.
"""
from __future__ import annotations

import numpy as np

__all__ = ["project", "interpolate", "tvir_of_expansion"]


def project(TT: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Least-squares coefficients per lag row.

    ``TT``: ``n x n`` TVIR matrix (row = lag, column = position);
    ``W``: ``m x n`` windows.  Returns ``h`` (``m x n``) with
    ``h[k, l] = c_k(lam(l)) / n``.
    """
    n = TT.shape[1]
    gram = W @ W.T                          # m x m
    rhs = W @ TT.T                          # m x n_lags
    c = np.linalg.solve(gram, rhs)          # c[k, l]
    return c / n


def interpolate(TT: np.ndarray, W: np.ndarray, node_cols) -> np.ndarray:
    """Interpolating coefficients at the node columns ``node_cols``."""
    n = TT.shape[1]
    E = W[:, node_cols].T                   # E[i, k] = w_k(y_i)
    c = np.linalg.solve(E, TT[:, node_cols].T)  # c[k, l]
    return c / n


def tvir_of_expansion(h: np.ndarray, W: np.ndarray) -> np.ndarray:
    """``T_m[l, j] = n sum_k h_k[l] w_k[j]`` (eq. 3.8 on the grid, rescaled to
    TVIR units so that it compares with ``TT``)."""
    n = W.shape[1]
    return n * (h.T @ W)
