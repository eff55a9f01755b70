"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's formula: each compares it with a
printed value, a closed form, a special case, an invariant, or a second
independent evaluation.
"""
import numpy as np
import pytest

from oracle import construct, dense, expansion as ex, grads
import workloads as wl


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ---------------------------------------------------------------------------
# Figure 1: the kernel builders reproduce the printed singular values
# ---------------------------------------------------------------------------

def _fig1_matrix(T, n=256):
    # Reading of Figure 1: points x_i = y_j = i/n - 1/2 and the matrix
    # sqrt(2) T(x_i, y_j) / n (the sqrt(2) is the printed scale; the ratios
    # below do not depend on it).
    x = np.arange(n) / n - 0.5
    return np.sqrt(2.0) * T(x[:, None], np.broadcast_to(x[None, :], (n, n))) / n


def test_fig1_spectrum1(golden):
    ref = np.array(golden("fig1_spectrum1.txt"))
    s = np.linalg.svd(_fig1_matrix(wl.tvir_gaussian(wl.example1_sigma)), compute_uv=False)
    np.testing.assert_allclose(s[:3], ref[:3], rtol=1e-9)
    np.testing.assert_allclose(s[3:6], ref[3:6], rtol=1e-5)
    # scale-free: the decay ratios pin the sigma-dependent normalisation
    np.testing.assert_allclose(s[1:3] / s[0], ref[1:3] / ref[0], rtol=1e-9)


def test_fig1_spectrum3_rank_two(golden):
    ref = np.array(golden("fig1_spectrum3.txt"))
    s = np.linalg.svd(_fig1_matrix(wl.example3_tvir(0.05, 0.1)), compute_uv=False)
    np.testing.assert_allclose(s[:2], ref[:2], rtol=1e-9)
    assert s[2] < 1e-13 * s[0]


def test_unnormalised_gaussian_fails_fig1(golden):
    # A plausible mistake (dropping 1/sigma) must not pass the pin.
    ref = np.array(golden("fig1_spectrum3.txt"))
    def T(x, y):
        yc = y - np.floor(y + 0.5)
        ind = (np.abs(yc) <= 0.25)
        g = lambda s: np.exp(-x * x / (2 * s * s)) / np.sqrt(2 * np.pi)  # noqa: E731
        return g(0.05) * ind + g(0.1) * (1 - ind)
    s = np.linalg.svd(_fig1_matrix(T), compute_uv=False)
    assert abs(s[1] / s[0] - ref[1] / ref[0]) > 1e-3


# ---------------------------------------------------------------------------
# B-spline windows (definition in the notation section)
# ---------------------------------------------------------------------------

def test_bspline_closed_forms_match_recurrence():
    # B_a = m B_0 * B_{a-1}: integrate the indicator against the previous
    # spline by a fine midpoint rule and compare with the closed forms.
    t = np.linspace(-2.5, 2.5, 501)
    s = np.linspace(-0.5, 0.5, 20001)[:-1] + 0.5 / 20000
    ds = 1.0 / 20000
    for deg in (1, 2, 3):
        prev = lambda x: wl.bspline_centered(x, deg - 1)  # noqa: E731
        num = np.array([np.sum(prev(ti - s)) * ds for ti in t])
        np.testing.assert_allclose(num, wl.bspline_centered(t, deg), atol=2e-4)


def test_cubic_knot_values_and_partition_of_unity():
    np.testing.assert_allclose(wl.bspline_centered(np.array([-1.0, 0.0, 1.0]), 3),
                               [1 / 6, 2 / 3, 1 / 6], rtol=0, atol=1e-15)
    for deg, m, n in ((1, 8, 1024), (3, 32, 4096), (1, 3, 384), (1, 2, 128), (3, 8, 96)):
        w = wl.bspline_windows_1d(n, m, deg)
        np.testing.assert_allclose(w.sum(0), 1.0, atol=1e-14)
    w = wl.tile_windows_1d(2048, 8)
    np.testing.assert_array_equal(w.sum(0), 1.0)


# ---------------------------------------------------------------------------
# The convolution of section 3.5: direction, sign, cross-agreement
# ---------------------------------------------------------------------------

FORMS = [(ex.apply_direct, ex.adjoint_direct), (ex.apply_dft, ex.adjoint_dft),
         (ex.apply_fft, ex.adjoint_fft)]


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_delta_input_gives_shifted_response(fwd, adj):
    n, j0 = 64, 5
    rng = np.random.default_rng(0)
    h = rng.standard_normal((1, n))
    u = np.zeros(n)
    u[j0] = 1.0
    y = fwd(u, np.ones((1, n)), h)
    np.testing.assert_allclose(y, np.roll(h[0], j0), atol=1e-12)
    # the adjoint of a shift-by-j0 convolution correlates: delta at i0 maps
    # to h[i0 - j] as a function of j
    v = np.zeros(n)
    v[j0] = 1.0
    x = adj(v, np.ones((1, n)), h)
    np.testing.assert_allclose(x, h[0][(j0 - np.arange(n)) % n], atol=1e-12)


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_geometric_filter_eigenvalue_closed_form(fwd, adj):
    # h[l] = a^l (l = 0..n-1) has DFT (1 - a^n) / (1 - a e^{-2 i pi f/n}); a
    # cosine of frequency f is mapped to Re(Hh[f] e^{2 i pi f t/n}).
    n, a, f = 96, 0.9, 7
    h = a ** np.arange(n)
    t = np.arange(n)
    hh = (1 - a ** n) / (1 - a * np.exp(-2j * np.pi * f / n))
    u = np.cos(2 * np.pi * f * t / n)
    y = fwd(u, np.ones((1, n)), h[None])
    np.testing.assert_allclose(y, np.real(hh * np.exp(2j * np.pi * f * t / n)), atol=1e-12)
    # adjoint: correlation uses conj(Hh)
    x = adj(u, np.ones((1, n)), h[None])
    np.testing.assert_allclose(x, np.real(np.conj(hh) * np.exp(2j * np.pi * f * t / n)), atol=1e-12)


def test_three_forms_agree_1d():
    p = wl.small_1d(256, 6, 3, batch=3, seed=11, sigma_fn=lambda y: 0.02 + 0.01 * y)
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    y0 = ex.apply_direct(u, w, h)
    assert _rel(ex.apply_dft(u, w, h), y0) < 1e-13
    assert _rel(ex.apply_fft(u, w, h), y0) < 1e-13
    x0 = ex.adjoint_direct(u, w, h)
    assert _rel(ex.adjoint_dft(u, w, h), x0) < 1e-13
    assert _rel(ex.adjoint_fft(u, w, h), x0) < 1e-13


def test_three_forms_agree_2d():
    p = wl.small_2d(16, 24, 2, 3, batch=2, seed=12)
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    y0 = ex.apply_direct(u, w, h)
    assert _rel(ex.apply_dft(u, w, h), y0) < 1e-13
    assert _rel(ex.apply_fft(u, w, h), y0) < 1e-13
    x0 = ex.adjoint_direct(u, w, h)
    assert _rel(ex.adjoint_dft(u, w, h), x0) < 1e-13
    assert _rel(ex.adjoint_fft(u, w, h), x0) < 1e-13


def test_2d_delta_shift():
    n1, n2 = 12, 10
    rng = np.random.default_rng(3)
    h = rng.standard_normal((1, n1, n2))
    u = np.zeros((n1, n2))
    u[3, 7] = 1.0
    for fwd, _ in FORMS:
        y = fwd(u, np.ones((1, n1, n2)), h)
        np.testing.assert_allclose(y, np.roll(h[0], (3, 7), axis=(0, 1)), atol=1e-12)


def test_sampled_direct_matches_full():
    p = wl.small_1d(512, 8, 3, batch=1, seed=5, sigma_fn=lambda y: 0.003 + 0.004 * y)
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u[0].astype(np.float64)
    assert np.sum(h == 0) > 0  # exact float32 zeros are skipped
    idx = np.array([0, 1, 77, 255, 256, 511])
    np.testing.assert_allclose(ex.apply_direct_at(u, w, h, idx),
                               ex.apply_direct(u, w, h)[idx], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(ex.adjoint_direct_at(u, w, h, idx),
                               ex.adjoint_direct(u, w, h)[idx], rtol=1e-13, atol=1e-15)
    q = wl.small_2d(32, 40, 2, 2, batch=1, seed=6)
    w2, h2, u2 = q.dense_windows(), q.h.astype(np.float64), q.u[0].astype(np.float64)
    idx2 = np.array([0, 5, 39, 40, 600, 32 * 40 - 1])
    np.testing.assert_allclose(ex.apply_direct_at(u2, w2, h2, idx2),
                               ex.apply_direct(u2, w2, h2).ravel()[idx2], rtol=1e-13)
    np.testing.assert_allclose(ex.adjoint_direct_at(u2, w2, h2, idx2),
                               ex.adjoint_direct(u2, w2, h2).ravel()[idx2], rtol=1e-13)


# ---------------------------------------------------------------------------
# Fixed points of the expansion
# ---------------------------------------------------------------------------

def test_m1_invariant_kernel_is_plain_convolution():
    # m = 1, w = 1 and a spatially invariant kernel: H_m = H, and both equal
    # the textbook circular convolution.
    n = 200
    T = wl.tvir_gaussian(lambda y: 0.03 + 0 * y)
    K = dense.kernel_matrix_1d(T, n)
    h = wl.sample_h_1d(T, n, [0.0])
    u = np.random.default_rng(4).standard_normal(n)
    y = ex.apply_direct(u, np.ones((1, n)), h)
    np.testing.assert_allclose(y, dense.apply_dense(K, u), rtol=1e-13, atol=1e-15)
    # the same convolution as a sum of shifted copies of u
    y2 = sum(h[0][l] * np.roll(u, l) for l in range(n))
    np.testing.assert_allclose(y, y2, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("deg,m", [(1, 8), (3, 16), (0, 4)])
def test_partition_of_unity_with_one_filter_is_a_convolution(deg, m):
    n = 256
    w = wl.bspline_windows_1d(n, m, deg) if deg > 0 else wl.tile_windows_1d(n, m)
    rng = np.random.default_rng(deg)
    h1 = rng.standard_normal(n)
    u = rng.standard_normal(n)
    y = ex.apply_direct(u, w, np.repeat(h1[None], m, 0))
    np.testing.assert_allclose(y, sum(h1[l] * np.roll(u, l) for l in range(n)),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_adjoint_identity(fwd, adj):
    p = wl.small_1d(240, 5, 3, batch=1, seed=8, sigma_fn=lambda y: 0.02 + 0.02 * y)
    w, h = p.dense_windows(), p.h.astype(np.float64)
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal(240), rng.standard_normal(240)
    hu, hv = fwd(u, w, h), adj(v, w, h)
    err = abs(np.dot(hu, v) - np.dot(u, hv)) / (np.linalg.norm(hu) * np.linalg.norm(v))
    assert err < 1e-12
    q = wl.small_2d(12, 16, 2, 2, seed=10)
    w2, h2 = q.dense_windows(), q.h.astype(np.float64)
    u2, v2 = rng.standard_normal((12, 16)), rng.standard_normal((12, 16))
    a, b = fwd(u2, w2, h2), adj(v2, w2, h2)
    err = abs(np.sum(a * v2) - np.sum(u2 * b)) / (np.linalg.norm(a) * np.linalg.norm(v2))
    assert err < 1e-12


def test_example3_two_terms_are_exact():
    # Example 3.3 is a sum of two tensor products: with the two indicator
    # windows and the two Gaussians as filters, H_2 = H to rounding.
    n = 512
    T = wl.example3_tvir(0.05, 0.1)
    K = dense.kernel_matrix_1d(T, n)
    y = np.arange(n) / n
    yc = y - np.floor(y + 0.5)
    w1 = (np.abs(yc) <= 0.25).astype(float)
    w = np.stack([w1, 1 - w1])
    lam = wl.lag_unit(n)
    h = np.stack([wl.gaussian(lam, 0.05), wl.gaussian(lam, 0.1)]) / n
    u = np.random.default_rng(12).standard_normal(n)
    np.testing.assert_allclose(ex.apply_direct(u, w, h), dense.apply_dense(K, u),
                               rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ex.adjoint_direct(u, w, h), dense.adjoint_dense(K, u),
                               rtol=1e-12, atol=1e-14)


def _shifted_two_tile_tvir(n):
    # A TVIR that is not symmetric in the lag: two Gaussians centred at
    # opposite nonzero lags, switched by the indicator of |y| <= 1/4 as in
    # Example 3.3.  Each column of the kernel is then a bump displaced from
    # the diagonal, in a direction fixed by the introduction's
    # K(x, y) = T(x - y, y).
    d1, d2 = 0.1, -0.07
    def T(x, y):
        yc = y - np.floor(np.asarray(y, np.float64) + 0.5)
        ind = (np.abs(yc) <= 0.25).astype(np.float64)
        return wl.gaussian(x - d1, 0.05) * ind + wl.gaussian(x - d2, 0.08) * (1.0 - ind)
    y = np.arange(n) / n
    yc = y - np.floor(y + 0.5)
    w1 = (np.abs(yc) <= 0.25).astype(float)
    lam = wl.lag_unit(n)
    h = np.stack([wl.gaussian(lam - d1, 0.05), wl.gaussian(lam - d2, 0.08)]) / n
    return T, np.stack([w1, 1 - w1]), h, (d1, d2)


def test_dense_quadrature_lag_direction():
    # The dense quadrature must put the response of the source y_j at
    # x_i = y_j + lag, i.e. K[i, j] = T(lam(i - j), y_j) / n.  With a TVIR
    # that is asymmetric in the lag and exactly two tensor products, the
    # two-term expansion with the centre-sampled shifted responses equals the
    # dense operator column by column (Lemma 3.1 with exact windows); a lag
    # taken as j - i would move every bump to the other side of the diagonal.
    n = 256
    T, w, h, (d1, d2) = _shifted_two_tile_tvir(n)
    K = dense.kernel_matrix_1d(T, n)
    for j in (0, 17, 64, 100, 128, 191, 255):
        e = np.zeros(n)
        e[j] = 1.0
        col = ex.apply_direct(e, w, h)
        np.testing.assert_allclose(col, K[:, j], rtol=1e-12, atol=1e-15)
        # the peak of column j sits at the index of y_j + d (mod 1)
        d = d1 if abs(j / n - np.floor(j / n + 0.5)) <= 0.25 else d2
        assert int(np.argmax(K[:, j])) == int(round((j / n + d) * n)) % n
    u = np.random.default_rng(31).standard_normal(n)
    np.testing.assert_allclose(ex.apply_direct(u, w, h), dense.apply_dense(K, u), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ex.adjoint_direct(u, w, h), dense.adjoint_dense(K, u), rtol=1e-12, atol=1e-14)
    # the test separates the two lag directions: the mirrored quadrature
    # differs from the expansion by the size of the operator itself
    i = np.arange(n)
    K_mirror = T(dense.lag_of(i[None, :] - i[:, None], n), np.broadcast_to((i / n)[None, :], (n, n))) / n
    assert _rel(K_mirror, K) > 0.5


def test_tvir_matrix_rows_are_lags():
    # tvir_matrix_1d's row l is the lag lam(l): with the shifted TVIR the
    # largest entry of each column sits at the row of the shift.
    n = 256
    T, _, _, (d1, d2) = _shifted_two_tile_tvir(n)
    TT = dense.tvir_matrix_1d(T, n)
    assert int(np.argmax(TT[:, 0])) == int(round(d1 * n)) % n
    assert int(np.argmax(TT[:, n // 2])) == int(round(d2 * n)) % n
    # and the kernel matrix is the TVIR read along the circulant diagonals
    K = dense.kernel_matrix_1d(T, n)
    for j in (0, 40, 128, 200):
        np.testing.assert_allclose(np.roll(K[:, j], -j), TT[:, j] / n, rtol=1e-13, atol=1e-16)


def test_hat_windows_interpolate_columns_at_centres():
    # Lemma 3.1 with interpolating hat windows: at a window centre y_j = c_k
    # only w_k is nonzero (and equals 1), so column j of H_m is column j of H.
    p = wl.config_c1()
    n, m = 1024, 8
    w = wl.bspline_windows_1d(n, m, 1)
    h = wl.sample_h_1d(p.T, n, np.arange(m) / m)
    K = dense.kernel_matrix_1d(p.T, n)
    for k in range(m):
        j = k * n // m
        e = np.zeros(n)
        e[j] = 1.0
        np.testing.assert_allclose(ex.apply_direct(e, w, h), K[:, j], rtol=1e-13, atol=1e-16)


def test_lemma_tvir_is_rank_m():
    # Lemma 3.1: the TVIR of the convolution-product expansion is
    # sum_k h_k(x) w_k(y).  Build H_m column by column from unit inputs.
    n, m = 64, 4
    rng = np.random.default_rng(13)
    w = rng.uniform(0, 1, (m, n))
    h = rng.standard_normal((m, n))
    cols = np.stack([ex.apply_direct(np.eye(n)[j], w, h) for j in range(n)], axis=1)
    tvir = np.stack([np.roll(cols[:, j], -j) for j in range(n)], axis=1)  # T[l, j] = K[l + j, j]
    np.testing.assert_allclose(tvir, h.T @ w, rtol=1e-12, atol=1e-13)
    s = np.linalg.svd(tvir, compute_uv=False)
    assert s[m] < 1e-12 * s[0]


def test_hs_norm_equals_tvir_norm():
    n = 128
    T = wl.tvir_gaussian(wl.example1_sigma)
    K = dense.kernel_matrix_1d(T, n)
    TT = dense.tvir_matrix_1d(T, n)
    assert abs(dense.hs_norm(K) - dense.hs_norm(TT) / n) < 1e-12 * dense.hs_norm(K)


# ---------------------------------------------------------------------------
# Approximation rates (sections 4.2 and 4.4)
# ---------------------------------------------------------------------------

def _slope(ms, errs):
    return float(np.polyfit(np.log(ms), np.log(errs), 1)[0])


def _proj_errors(sigma_fn, deg, ms, n=1024):
    T = wl.tvir_gaussian(sigma_fn)
    TT = dense.tvir_matrix_1d(T, n)
    out = []
    for m in ms:
        W = wl.bspline_windows_1d(n, m, deg)
        h = construct.project(TT, W)
        out.append(_rel(construct.tvir_of_expansion(h, W), TT))
    return out


@pytest.mark.parametrize("deg", [1, 3])
def test_projection_rate_smooth_kernel(deg):
    # Corollary 4.3: for T(x, .) in H^s and degree >= s the HS error decays at
    # least like m^{-s}; Example 3.1 width field is smooth, so s = degree.
    ms = [8, 16, 32, 64]
    errs = _proj_errors(wl.example1_sigma, deg, ms)
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert _slope(ms, errs) <= -deg + 0.1


def test_projection_rate_rough_kernel():
    # sigma(y) = 0.01 + 0.02 y jumps at the periodic wrap: T(x, .) is in H^s
    # only for s < 1/2, so only a rate close to m^{-1/2} is available.
    ms = [8, 16, 32, 64, 128]
    errs = _proj_errors(lambda y: 0.01 + 0.02 * y, 1, ms)
    sl = _slope(ms, errs)
    assert -0.75 < sl <= -0.4


def test_interpolation_with_hat_windows_is_centre_sampling():
    n, m = 256, 8
    T = wl.tvir_gaussian(wl.example1_sigma)
    TT = dense.tvir_matrix_1d(T, n)
    W = wl.bspline_windows_1d(n, m, 1)
    nodes = [k * n // m for k in range(m)]
    h = construct.interpolate(TT, W, nodes)
    np.testing.assert_allclose(h, wl.sample_h_1d(T, n, np.arange(m) / m), rtol=1e-13)


# ---------------------------------------------------------------------------
# Gradients (finite differences on the FFT form)
# ---------------------------------------------------------------------------

def _loss_from_spectra(hs, wz_hat, f, shape):
    import scipy.fft as sfft
    nd = len(shape)
    y = sfft.irfftn(np.sum(hs * wz_hat, axis=0), s=shape, axes=tuple(range(-nd, 0)))
    return 0.5 * np.sum((y - f) ** 2)


@pytest.mark.parametrize("shape", [(32,), (8, 12)])
def test_grad_spectra_finite_differences(shape):
    import scipy.fft as sfft
    rng = np.random.default_rng(14)
    m = 3
    nd = len(shape)
    axes = tuple(range(-nd, 0))
    w = rng.uniform(0, 1, (m,) + shape)
    h = rng.standard_normal((m,) + shape)
    u = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    hs = sfft.rfftn(h, axes=axes)
    wz = sfft.rfftn(w * u[None], axes=axes)
    y = sfft.irfftn(np.sum(hs * wz, 0), s=shape, axes=axes)
    g = y - f
    G = grads.grad_spectra(u[None], g[None], w)
    eps = 1e-6
    last = shape[-1] // 2
    bins = [(0,) * nd, (0,) * (nd - 1) + (last,), (0,) * (nd - 1) + (1,)]
    if nd == 2:
        bins += [(3, 0), (5, last), (2, 4)]
    for k in range(m):
        for b in bins:
            for part in (1.0, 1j):
                hp = hs.copy()
                hm = hs.copy()
                hp[(k,) + b] += eps * part
                hm[(k,) + b] -= eps * part
                fd = (_loss_from_spectra(hp, wz, f, shape) - _loss_from_spectra(hm, wz, f, shape)) / (2 * eps)
                an = G[(k,) + b].real if part == 1.0 else G[(k,) + b].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (k, b, part, fd, an)


def test_grad_u_finite_differences():
    rng = np.random.default_rng(15)
    n, m = 48, 3
    w = rng.uniform(0, 1, (m, n))
    h = rng.standard_normal((m, n))
    u = rng.standard_normal(n)
    f = rng.standard_normal(n)
    g = ex.apply_fft(u, w, h) - f
    gu = grads.grad_u(g, w, h)
    d = rng.standard_normal(n)
    eps = 1e-6
    L = lambda x: 0.5 * np.sum((ex.apply_fft(x, w, h) - f) ** 2)  # noqa: E731
    fd = (L(u + eps * d) - L(u - eps * d)) / (2 * eps)
    assert abs(fd - np.dot(gu, d)) < 1e-7 * abs(fd)
