"""Pins of the wavelet oracle and of Meyer's operator representation
(section 4.5): the published closed form of the 4-tap Daubechies filter, the
filter identities (sum, orthogonality to even shifts, vanishing moments),
orthogonality of the DWT matrix, the explicit Haar matrix, perfect
reconstruction of the TVIR from all its coefficients, Parseval for
truncations, and the regrouping of the trick equation against the term-by-term
double sum."""
import numpy as np
import pytest

import workloads as wl
from oracle import construct, dense, expansion as ex, wavelets as wv


def test_db2_closed_form():
    s3 = np.sqrt(3.0)
    want = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    np.testing.assert_allclose(wv.daubechies(2), want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_filter_identities(N):
    h = wv.daubechies(N)
    assert h.shape == (2 * N,)
    assert abs(np.sum(h) - np.sqrt(2.0)) < 1e-12
    for j in range(N):
        assert abs(np.dot(h[:len(h) - 2 * j], h[2 * j:]) - (1.0 if j == 0 else 0.0)) < 1e-12
    g = np.array([(-1) ** k * h[len(h) - 1 - k] for k in range(len(h))])
    k = np.arange(len(h))
    for p in range(N):
        assert abs(np.sum(k ** p * g)) < 1e-9 * max(1, len(h) ** p)


@pytest.mark.parametrize("N,n,levels", [(1, 16, 4), (2, 32, 3), (3, 64, 4), (4, 64, 2)])
def test_dwt_matrix_is_orthogonal(N, n, levels):
    P = wv.dwt_matrix(n, wv.daubechies(N), levels)
    np.testing.assert_allclose(P @ P.T, np.eye(n), atol=1e-12)
    x = np.random.default_rng(N).standard_normal((2, n))
    np.testing.assert_allclose(wv.idwt(wv.dwt(x, wv.daubechies(N), levels), wv.daubechies(N), levels), x,
                               atol=1e-12)


def test_haar_matrix_explicit():
    r = 1 / np.sqrt(2.0)
    want = np.array([[0.5, 0.5, 0.5, 0.5], [0.5, 0.5, -0.5, -0.5], [r, -r, 0, 0], [0, 0, r, -r]])
    np.testing.assert_allclose(wv.dwt_matrix(4, wv.daubechies(1), 2), want, atol=1e-15)


def _tvir(n):
    return dense.tvir_matrix_1d(wl.tvir_gaussian(lambda y: 0.03 + 0.02 * np.sin(2 * np.pi * y)), n)


def test_all_coefficients_reconstruct_the_tvir():
    n, levels = 64, 4
    h = wv.daubechies(3)
    TT = _tvir(n)
    C = wv.meyer_coefficients(TT, h, levels)
    lam, mu = np.nonzero(np.ones_like(C))
    mus, w, hk = wv.meyer_expansion(lam, mu, C[lam, mu], n, h, levels)
    assert mus.shape[0] == n
    np.testing.assert_allclose(construct.tvir_of_expansion(hk, w), TT, atol=1e-10 * np.abs(TT).max())


def test_truncation_error_is_parseval():
    n, levels = 64, 4
    h = wv.daubechies(2)
    TT = _tvir(n)
    C = wv.meyer_coefficients(TT, h, levels)
    keep = np.argsort(np.abs(C).ravel())[::-1][:300]
    lam, mu = np.unravel_index(keep, C.shape)
    _, w, hk = wv.meyer_expansion(lam, mu, C[lam, mu], n, h, levels)
    Cs = np.zeros_like(C)
    Cs[lam, mu] = C[lam, mu]
    err = np.linalg.norm(construct.tvir_of_expansion(hk, w) - TT)
    assert abs(err - np.linalg.norm(C - Cs)) < 1e-10 * np.linalg.norm(TT)


def test_trick_equation_regrouping():
    # sum_{lam,mu} c psi_lam * (psi_mu . u) / n, term by term, against the
    # expansion regrouped by mu
    n, levels = 32, 3
    h = wv.daubechies(2)
    rng = np.random.default_rng(5)
    lam = rng.integers(0, n, 40)
    mu = rng.integers(0, 6, 40)
    c = rng.standard_normal(40)
    u = rng.standard_normal(n)
    P = wv.dwt_matrix(n, h, levels)
    direct = np.zeros(n)
    for a, b, v in zip(lam, mu, c):
        direct += ex.apply_direct(u, P[b][None], (v * P[a] / n)[None])
    _, w, hk = wv.meyer_expansion(lam, mu, c, n, h, levels)
    np.testing.assert_allclose(ex.apply_fft(u, w, hk), direct, atol=1e-12)
