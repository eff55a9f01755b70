"""The convolution-product expansion, evaluated plainly in float64.

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the bench's
CPU baseline.

Definitions followed (section numbers of the paper):

* eq. (1.4): ``H_m u = sum_{k=1..m} h_k * (w_k . u)``.
* section 3.5: the discrete circular convolution
  ``v[i] = sum_j u[i - j] h[j]`` (indices mod n; written 0-based here, index
  0 of ``h`` is the zero lag), and the identity
  ``v = F_n ((F_n^* h) . (F_n^* u))`` with ``F_n^*`` the DFT and ``F_n`` its
  inverse.  The DFT uses the Fourier atoms of the notation section,
  ``exp(-2 i pi k x)``, so ``(F^* x)[f] = sum_n x[n] exp(-2 i pi f n / N)``
  and ``F = conj(F^*)^T / N``.
* The adjoint of a real expansion: ``H_m^* v = sum_k w_k . (h~_k * v)``
  with ``h~_k[l] = h_k[-l]``, i.e. ``(H_m^* v)[j] = sum_k w_k[j]
  sum_i h_k[i - j] v[i]``.
* eq. (1.3), the product-convolution expansion (the ``*_pc_*`` functions):
  ``G_m u = sum_k w_k . (h_k * u)``, i.e. ``(G_m u)[i] = sum_k w_k[i]
  sum_j h_k[i - j] u[j]``, and its adjoint ``G_m^* v = sum_k h~_k *
  (w_k . v)``, i.e. ``(G_m^* v)[j] = sum_k sum_i h_k[i - j] w_k[i] v[i]``.

2D uses the same formulas with index pairs taken modulo ``(N1, N2)``.
Inputs are real (``u``, ``w_k``, ``h_k``); the functions accept a single
signal (``N`` or ``N1 x N2``) or a leading batch axis.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

__all__ = [
    "apply_direct", "adjoint_direct", "apply_direct_at", "adjoint_direct_at",
    "apply_dft", "adjoint_dft", "apply_fft", "adjoint_fft", "workers",
    "dft_matrix",
    "apply_pc_direct", "adjoint_pc_direct", "apply_pc_direct_at", "adjoint_pc_direct_at",
    "apply_pc_fft", "adjoint_pc_fft",
]


def workers() -> int:
    """Threads the FFT-library form may use (the cores this process may run on)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _batched(u, ndim):
    u = np.asarray(u, dtype=np.float64)
    single = u.ndim == ndim
    return (u[None] if single else u), single


# ----------------------------------------------------------------------------
# O2: direct circular sums (the plain definition)
# ----------------------------------------------------------------------------

def _circulant(h: np.ndarray) -> np.ndarray:
    """Matrix ``C[i, j] = h[(i - j) mod N]`` (1D) or the block-circulant
    matrix over flattened index pairs (2D)."""
    if h.ndim == 1:
        n = h.shape[0]
        i = np.arange(n)
        return h[(i[:, None] - i[None, :]) % n]
    n1, n2 = h.shape
    i1 = np.arange(n1)
    i2 = np.arange(n2)
    d1 = (i1[:, None] - i1[None, :]) % n1           # [i1, j1]
    d2 = (i2[:, None] - i2[None, :]) % n2           # [i2, j2]
    c = h[d1[:, None, :, None], d2[None, :, None, :]]  # [i1, i2, j1, j2]
    return c.reshape(n1 * n2, n1 * n2)


def apply_direct(u, w, h):
    """``H_m u`` by direct sums; ``O(m N^2)`` — tiny grids only."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    ub, single = _batched(u, nd)
    out = np.zeros_like(ub)
    for k in range(w.shape[0]):
        c = _circulant(h[k])
        z = (w[k][None] * ub).reshape(ub.shape[0], -1)
        out += (z @ c.T).reshape(ub.shape)
    return out[0] if single else out


def adjoint_direct(v, w, h):
    """``H_m^* v`` by direct sums: ``sum_k w_k[j] sum_i h_k[i-j] v[i]``."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    vb, single = _batched(v, nd)
    out = np.zeros_like(vb)
    flat = vb.reshape(vb.shape[0], -1)
    for k in range(w.shape[0]):
        c = _circulant(h[k])
        g = (flat @ c).reshape(vb.shape)      # sum_i C[i, j] v[i]
        out += w[k][None] * g
    return out[0] if single else out


def _support_lags(hk: np.ndarray):
    """Indices where the impulse response is nonzero (exact zeros skipped,
    which changes no sum)."""
    return np.nonzero(hk)


def apply_direct_at(u, w, h, idx, chunk=256):
    """Selected outputs of ``H_m u`` by direct sums.

    ``u``: one signal (``N`` or ``N1 x N2``); ``idx``: array of flat output
    indices.  Each output is ``sum_k sum_l h_k[l] w_k[i - l] u[i - l]`` over
    the nonzero lags ``l`` of ``h_k``; this is the definition with the
    substitution ``j = i - l``.
    """
    u = np.asarray(u, np.float64)
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    shape = u.shape
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[0])
    if len(shape) == 1:
        n = shape[0]
        for k in range(w.shape[0]):
            (ls,) = _support_lags(h[k])
            hv = h[k][ls]
            z = w[k] * u
            for s in range(0, idx.shape[0], chunk):
                ii = idx[s:s + chunk]
                out[s:s + chunk] += z[(ii[:, None] - ls[None, :]) % n] @ hv
    else:
        n1, n2 = shape
        i1, i2 = np.unravel_index(idx, shape)
        for k in range(w.shape[0]):
            l1, l2 = _support_lags(h[k])
            hv = h[k][l1, l2]
            z = w[k] * u
            for s in range(0, idx.shape[0], chunk):
                a = i1[s:s + chunk, None]
                b = i2[s:s + chunk, None]
                out[s:s + chunk] += z[(a - l1[None]) % n1, (b - l2[None]) % n2] @ hv
    return out


def adjoint_direct_at(v, w, h, idx, chunk=256):
    """Selected outputs of ``H_m^* v``: ``w_k[j] sum_l h_k[l] v[j + l]``."""
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    shape = v.shape
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[0])
    if len(shape) == 1:
        n = shape[0]
        for k in range(w.shape[0]):
            (ls,) = _support_lags(h[k])
            hv = h[k][ls]
            for s in range(0, idx.shape[0], chunk):
                jj = idx[s:s + chunk]
                out[s:s + chunk] += w[k][jj] * (v[(jj[:, None] + ls[None, :]) % n] @ hv)
    else:
        n1, n2 = shape
        j1, j2 = np.unravel_index(idx, shape)
        for k in range(w.shape[0]):
            l1, l2 = _support_lags(h[k])
            hv = h[k][l1, l2]
            for s in range(0, idx.shape[0], chunk):
                a = j1[s:s + chunk]
                b = j2[s:s + chunk]
                g = v[(a[:, None] + l1[None]) % n1, (b[:, None] + l2[None]) % n2] @ hv
                out[s:s + chunk] += w[k][a, b] * g
    return out


# ----------------------------------------------------------------------------
# O2': explicit DFT matrices (section 3.5 written out)
# ----------------------------------------------------------------------------

def dft_matrix(n: int) -> np.ndarray:
    """``F^*[f, t] = exp(-2 i pi f t / n)`` (unnormalised DFT)."""
    f = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(f, f) / n)


def _dft_nd(x, mats):
    """Apply one DFT matrix per trailing axis (the 2D DFT is the double sum)."""
    if len(mats) == 1:
        return x @ mats[0].T
    a, b = mats
    return np.einsum("fi,...ij,gj->...fg", a, x, b, optimize=True)


def _idft_nd(x, mats):
    n = np.prod([m.shape[0] for m in mats])
    return _dft_nd(x, [np.conj(m) for m in mats]) / n


def apply_dft(u, w, h):
    """``H_m u = F (sum_k (F^* h_k) . (F^* (w_k . u)))`` with explicit matrices."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    ub, single = _batched(u, nd)
    mats = [dft_matrix(s) for s in h.shape[1:]]
    acc = np.zeros(ub.shape, dtype=np.complex128)
    for k in range(w.shape[0]):
        acc += _dft_nd(h[k], mats)[None] * _dft_nd(w[k][None] * ub, mats)
    out = _idft_nd(acc, mats).real
    return out[0] if single else out


def adjoint_dft(v, w, h):
    """``H_m^* v = sum_k w_k . F (conj(F^* h_k) . (F^* v))``."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    vb, single = _batched(v, nd)
    mats = [dft_matrix(s) for s in h.shape[1:]]
    vh = _dft_nd(vb, mats)
    out = np.zeros(vb.shape)
    for k in range(w.shape[0]):
        g = _idft_nd(np.conj(_dft_nd(h[k], mats))[None] * vh, mats).real
        out += w[k][None] * g
    return out[0] if single else out


# ----------------------------------------------------------------------------
# O2'': the same identity through a float64 FFT library (large sizes)
# ----------------------------------------------------------------------------

def _rfftn(x, nd):
    axes = tuple(range(-nd, 0))
    return sfft.rfftn(x, axes=axes, workers=workers())


def _irfftn(x, shape, nd):
    axes = tuple(range(-nd, 0))
    return sfft.irfftn(x, s=shape, axes=axes, workers=workers())


def apply_fft(u, w, h, h_spec=None):
    """``H_m u`` via float64 real FFTs.  ``h_spec`` may hold the precomputed
    half-spectra ``rfftn(h_k)`` (``m x ...``)."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    ub, single = _batched(u, nd)
    shape = ub.shape[1:]
    hs = _rfftn(np.asarray(h, np.float64), nd) if h_spec is None else h_spec
    acc = None
    for k in range(w.shape[0]):
        term = hs[k][None] * _rfftn(w[k][None] * ub, nd)
        acc = term if acc is None else acc + term
    out = _irfftn(acc, shape, nd)
    return out[0] if single else out


def adjoint_fft(v, w, h, h_spec=None):
    """``H_m^* v`` via float64 real FFTs."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    vb, single = _batched(v, nd)
    shape = vb.shape[1:]
    hs = _rfftn(np.asarray(h, np.float64), nd) if h_spec is None else h_spec
    vh = _rfftn(vb, nd)
    out = np.zeros(vb.shape)
    for k in range(w.shape[0]):
        out += w[k][None] * _irfftn(np.conj(hs[k])[None] * vh, shape, nd)
    return out[0] if single else out


# ----------------------------------------------------------------------------
# eq. (1.3): the product-convolution expansion, the same three ways
# ----------------------------------------------------------------------------

def apply_pc_direct(u, w, h):
    """``G_m u = sum_k w_k . (h_k * u)`` by direct sums; tiny grids only."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    ub, single = _batched(u, nd)
    flat = ub.reshape(ub.shape[0], -1)
    out = np.zeros_like(ub)
    for k in range(w.shape[0]):
        c = _circulant(h[k])
        out += w[k][None] * (flat @ c.T).reshape(ub.shape)
    return out[0] if single else out


def adjoint_pc_direct(v, w, h):
    """``G_m^* v = sum_k h~_k * (w_k . v)``: ``sum_k sum_i h_k[i-j] w_k[i] v[i]``."""
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    nd = h.ndim - 1
    vb, single = _batched(v, nd)
    out = np.zeros_like(vb)
    for k in range(w.shape[0]):
        c = _circulant(h[k])
        z = (w[k][None] * vb).reshape(vb.shape[0], -1)
        out += (z @ c).reshape(vb.shape)          # sum_i C[i, j] z[i]
    return out[0] if single else out


def apply_pc_direct_at(u, w, h, idx, chunk=256):
    """Selected outputs of ``G_m u``: ``w_k[i] sum_l h_k[l] u[i - l]`` over the
    nonzero lags ``l`` of ``h_k``."""
    u = np.asarray(u, np.float64)
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    shape = u.shape
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[0])
    if len(shape) == 1:
        n = shape[0]
        for k in range(w.shape[0]):
            (ls,) = _support_lags(h[k])
            hv = h[k][ls]
            for s in range(0, idx.shape[0], chunk):
                ii = idx[s:s + chunk]
                out[s:s + chunk] += w[k][ii] * (u[(ii[:, None] - ls[None, :]) % n] @ hv)
    else:
        n1, n2 = shape
        i1, i2 = np.unravel_index(idx, shape)
        for k in range(w.shape[0]):
            l1, l2 = _support_lags(h[k])
            hv = h[k][l1, l2]
            for s in range(0, idx.shape[0], chunk):
                a = i1[s:s + chunk]
                b = i2[s:s + chunk]
                g = u[(a[:, None] - l1[None]) % n1, (b[:, None] - l2[None]) % n2] @ hv
                out[s:s + chunk] += w[k][a, b] * g
    return out


def adjoint_pc_direct_at(v, w, h, idx, chunk=256):
    """Selected outputs of ``G_m^* v``: ``sum_k sum_l h_k[l] (w_k v)[j + l]``."""
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    h = np.asarray(h, np.float64)
    shape = v.shape
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[0])
    if len(shape) == 1:
        n = shape[0]
        for k in range(w.shape[0]):
            (ls,) = _support_lags(h[k])
            hv = h[k][ls]
            z = w[k] * v
            for s in range(0, idx.shape[0], chunk):
                jj = idx[s:s + chunk]
                out[s:s + chunk] += z[(jj[:, None] + ls[None, :]) % n] @ hv
    else:
        n1, n2 = shape
        j1, j2 = np.unravel_index(idx, shape)
        for k in range(w.shape[0]):
            l1, l2 = _support_lags(h[k])
            hv = h[k][l1, l2]
            z = w[k] * v
            for s in range(0, idx.shape[0], chunk):
                a = j1[s:s + chunk, None]
                b = j2[s:s + chunk, None]
                out[s:s + chunk] += z[(a + l1[None]) % n1, (b + l2[None]) % n2] @ hv
    return out


def apply_pc_fft(u, w, h, h_spec=None):
    """``G_m u`` via float64 real FFTs: ``sum_k w_k . F((F^* h_k) . (F^* u))``."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    ub, single = _batched(u, nd)
    shape = ub.shape[1:]
    hs = _rfftn(np.asarray(h, np.float64), nd) if h_spec is None else h_spec
    uh = _rfftn(ub, nd)
    out = np.zeros(ub.shape)
    for k in range(w.shape[0]):
        out += w[k][None] * _irfftn(hs[k][None] * uh, shape, nd)
    return out[0] if single else out


def adjoint_pc_fft(v, w, h, h_spec=None):
    """``G_m^* v`` via float64 real FFTs: ``F(sum_k conj(F^* h_k) . F^*(w_k . v))``."""
    w = np.asarray(w, np.float64)
    nd = w.ndim - 1
    vb, single = _batched(v, nd)
    shape = vb.shape[1:]
    hs = _rfftn(np.asarray(h, np.float64), nd) if h_spec is None else h_spec
    acc = None
    for k in range(w.shape[0]):
        term = np.conj(hs[k])[None] * _rfftn(w[k][None] * vb, nd)
        acc = term if acc is None else acc + term
    out = _irfftn(acc, shape, nd)
    return out[0] if single else out
