"""Gradients of a scalar loss through ``y = H_m u`` (TEST INFRASTRUCTURE).

Imported only by tests and the bench's CPU baseline.

With ``y = irfftn(S)``, ``S = sum_k Hh_k . Z_k``, ``Z_k = rfftn(w_k . u)``
(the identity of section 3.5 written on half-spectra) and an upstream
gradient ``g = dL/dy``:

* ``dL/du = H_m^* g`` (the adjoint of eq. 1.4);
* for the half-spectrum ``Hh_k`` (complex gradient convention
  ``dL/dRe + i dL/dIm``): ``G_k = conj(Z_k) . c . rfftn(g) / N`` where
  ``N`` is the number of samples, ``c = 2`` on the bins of the last axis that
  stand for a conjugate pair and ``c = 1`` on its DC and (even-length)
  Nyquist bins, whose imaginary parts the inverse real transform discards.

For the product-convolution expansion of eq. (1.3), ``y = sum_k w_k .
irfftn(Hh_k . rfftn(u))``, the same computation with the pairing moved gives
``G_k = conj(rfftn(u)) . c . rfftn(w_k . g) / N``.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .expansion import adjoint_fft, workers

__all__ = ["half_weights", "grad_u", "grad_spectra", "grad_spectra_pc"]


def half_weights(n_last: int) -> np.ndarray:
    """``c`` over the ``n_last//2 + 1`` bins of the last axis."""
    c = np.full(n_last // 2 + 1, 2.0)
    c[0] = 1.0
    if n_last % 2 == 0:
        c[-1] = 1.0
    return c


def grad_u(g, w, h):
    """``dL/du = H_m^* g``."""
    return adjoint_fft(g, w, h)


def grad_spectra(u, g, w):
    """``dL/dHh_k`` summed over the batch.  ``u``, ``g``: ``B x shape``."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    u = np.asarray(u, np.float64).reshape((-1,) + w.shape[1:])
    g = np.asarray(g, np.float64).reshape(u.shape)
    axes = tuple(range(-nd, 0))
    ntot = int(np.prod(w.shape[1:]))
    c = half_weights(w.shape[-1])
    gh = sfft.rfftn(g, axes=axes, workers=workers()) * c / ntot
    out = []
    for k in range(w.shape[0]):
        zk = sfft.rfftn(w[k][None] * u, axes=axes, workers=workers())
        out.append(np.sum(np.conj(zk) * gh, axis=0))
    return np.stack(out)


def grad_spectra_pc(u, g, w):
    """``dL/dHh_k`` through the product-convolution expansion (eq. 1.3),
    summed over the batch.  ``u``, ``g``: ``B x shape``."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    u = np.asarray(u, np.float64).reshape((-1,) + w.shape[1:])
    g = np.asarray(g, np.float64).reshape(u.shape)
    axes = tuple(range(-nd, 0))
    ntot = int(np.prod(w.shape[1:]))
    c = half_weights(w.shape[-1])
    uh = np.conj(sfft.rfftn(u, axes=axes, workers=workers())) * c / ntot
    out = []
    for k in range(w.shape[0]):
        qk = sfft.rfftn(w[k][None] * g, axes=axes, workers=workers())
        out.append(np.sum(uh * qk, axis=0))
    return np.stack(out)
