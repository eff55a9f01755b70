"""Periodic orthonormal wavelets and Meyer's operator representation
(TEST INFRASTRUCTURE; imported only by tests and the bench's CPU baseline).

Section 4.5 ("On Meyer's operator representation") expands the TVIR in the
tensor basis psi_lambda (x) psi_mu and keeps m coefficients
c_{lambda,mu} = <T, psi_lambda (x) psi_mu>; regrouping the sum by mu (the
paper's trick equation) gives a convolution-product expansion with windows
w_mu = psi_mu and responses c~_mu = sum_lambda c_{lambda,mu} psi_lambda.

On a grid of n = 2^J samples the basis is the periodic orthonormal discrete
wavelet basis of a Daubechies filter: the rows of the matrix Psi of the
discrete wavelet transform (DWT), coefficients in pyramid order
[approximation at the coarsest level, details coarse to fine].  With the TVIR
matrix TT[l, j] (row = lag, column = position, as in `dense.tvir_matrix_1d`),
C = Psi TT Psi^T, and the expansion of a coefficient set is
    w_mu = Psi[mu, :],   h_mu = (Psi^T C[:, mu]) / n,
so that n sum_mu h_mu[l] w_mu[j] reconstructs sum C[lam, mu] Psi[lam, l] Psi[mu, j].

Daubechies filters (Daubechies 1988): the lowpass filter with N vanishing
moments is the spectral factor of |m0(w)|^2 = cos^{2N}(w/2) P(sin^2(w/2)),
P(y) = sum_{k<N} binom(N-1+k, k) y^k, keeping the roots inside the unit
circle; the highpass filter is g[k] = (-1)^k h[L-1-k].
"""
from __future__ import annotations

from math import comb

import numpy as np

__all__ = ["daubechies", "dwt", "idwt", "dwt_matrix", "meyer_coefficients", "meyer_expansion"]


def daubechies(N: int) -> np.ndarray:
    """Lowpass filter (length 2N, sum sqrt(2)) with N vanishing moments."""
    if N == 1:
        return np.array([1.0, 1.0]) / np.sqrt(2.0)
    # P(y) with y = sin^2(w/2) = (2 - z - 1/z)/4; roots of P in y map to pairs of z roots
    py = [comb(N - 1 + k, k) for k in range(N)]          # coefficients of y^k
    yr = np.roots(py[::-1])                              # roots in y
    zr = []
    for y in yr:
        # y = (2 - z - 1/z)/4  ->  z^2 - (2 - 4y) z + 1 = 0
        zz = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        zr.append(zz[np.argmin(np.abs(zz))])            # the root inside the unit circle
    poly = np.array([1.0])
    for _ in range(N):
        poly = np.convolve(poly, [1.0, 1.0])             # (1 + z^-1)^N
    for z in zr:
        poly = np.convolve(poly, [1.0, -z])
    h = np.real(poly)
    return h / np.sum(h) * np.sqrt(2.0)


def _highpass(h: np.ndarray) -> np.ndarray:
    L = h.shape[0]
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])


def _analysis_step(a: np.ndarray, h: np.ndarray):
    """One level on the last axis: approximation and detail, periodic:
    lo[i] = sum_k h[k] a[(2i + k) mod n],  hi[i] = sum_k g[k] a[(2i + k) mod n]."""
    n = a.shape[-1]
    g = _highpass(h)
    lo = np.zeros(a.shape[:-1] + (n // 2,))
    hi = np.zeros_like(lo)
    for k in range(h.shape[0]):
        v = a[..., (2 * np.arange(n // 2) + k) % n]
        lo += h[k] * v
        hi += g[k] * v
    return lo, hi


def _synthesis_step(lo: np.ndarray, hi: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Inverse of `_analysis_step` (its transpose, the step being orthogonal):
    out[(2i + k) mod n] += h[k] lo[i] + g[k] hi[i]."""
    half = lo.shape[-1]
    n = 2 * half
    g = _highpass(h)
    out = np.zeros(lo.shape[:-1] + (n,))
    for k in range(h.shape[0]):
        pos = (2 * np.arange(half) + k) % n      # distinct for a fixed k
        out[..., pos] += lo * h[k] + hi * g[k]
    return out


def dwt(x: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Periodic DWT over the last axis, pyramid order [a_J, d_J, ..., d_1]."""
    a = np.asarray(x, np.float64)
    details = []
    for _ in range(levels):
        a, d = _analysis_step(a, h)
        details.append(d)
    return np.concatenate([a] + details[::-1], axis=-1)


def idwt(c: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Inverse of `dwt`."""
    c = np.asarray(c, np.float64)
    n = c.shape[-1]
    size = n >> levels
    a = c[..., :size]
    pos = size
    for _ in range(levels):
        d = c[..., pos:pos + size]
        a = _synthesis_step(a, d, h)
        pos += size
        size *= 2
    return a


def dwt_matrix(n: int, h: np.ndarray, levels: int) -> np.ndarray:
    """Psi with dwt(x) = Psi x (rows: the basis vectors); `dwt` transforms
    each row of the identity, which gives Psi^T."""
    return dwt(np.eye(n), h, levels).T


def meyer_coefficients(TT: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """C[lam, mu] = <TT, psi_lam (x) psi_mu> = (Psi TT Psi^T)[lam, mu]."""
    return dwt(dwt(TT, h, levels).T, h, levels).T


def meyer_expansion(lam, mu, c, n: int, h: np.ndarray, levels: int):
    """Windows and responses of the expansion regrouped by mu (the trick
    equation): returns (mus, w, hk) with w[i] = psi_{mus[i]},
    hk[i] = (sum_lam c_{lam, mus[i]} psi_lam) / n."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    c = np.asarray(c, np.float64)
    mus = np.unique(mu)
    coef = np.zeros((mus.shape[0], n))
    e = np.zeros((mus.shape[0], n))
    for i, m_ in enumerate(mus):
        sel = mu == m_
        np.add.at(coef[i], lam[sel], c[sel])
        e[i, m_] = 1.0
    return mus, idwt(e, h, levels), idwt(coef, h, levels) / n
