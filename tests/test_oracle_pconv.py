"""Pins of the product-convolution oracle (eq. 1.3): G_m u = sum_k w_k . (h_k * u).

Each case checks the oracle against something fixed outside it: explicit
loops over the definition on tiny grids, closed forms (delta responses,
delta inputs, constant windows), the adjoint relation with the
convolution-product oracle on flipped responses, and finite differences of
the spectra gradient.
"""
import numpy as np
import pytest

from oracle import expansion as ex, grads


def _flip(h):
    """h~[l] = h[-l] on every axis (lag layout)."""
    out = np.asarray(h, np.float64)
    for ax in range(1, out.ndim):
        out = np.roll(np.flip(out, axis=ax), 1, axis=ax)
    return out


def _loops_1d(u, w, h):
    n = u.shape[0]
    y = np.zeros(n)
    for k in range(w.shape[0]):
        for i in range(n):
            s = 0.0
            for j in range(n):
                s += h[k][(i - j) % n] * u[j]
            y[i] += w[k][i] * s
    return y


def _loops_1d_adjoint(v, w, h):
    n = v.shape[0]
    x = np.zeros(n)
    for k in range(w.shape[0]):
        for j in range(n):
            for i in range(n):
                x[j] += h[k][(i - j) % n] * w[k][i] * v[i]
    return x


def _loops_2d(u, w, h):
    n1, n2 = u.shape
    y = np.zeros((n1, n2))
    for k in range(w.shape[0]):
        for i1 in range(n1):
            for i2 in range(n2):
                s = 0.0
                for j1 in range(n1):
                    for j2 in range(n2):
                        s += h[k][(i1 - j1) % n1, (i2 - j2) % n2] * u[j1, j2]
                y[i1, i2] += w[k][i1, i2] * s
    return y


FORMS = [(ex.apply_pc_direct, ex.adjoint_pc_direct), (ex.apply_pc_fft, ex.adjoint_pc_fft)]


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_loops_1d(fwd, adj):
    rng = np.random.default_rng(31)
    n, m = 11, 3
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    w = rng.uniform(0, 1, (m, n))
    h = rng.standard_normal((m, n))
    assert np.allclose(fwd(u, w, h), _loops_1d(u, w, h), rtol=0, atol=1e-12)
    assert np.allclose(adj(v, w, h), _loops_1d_adjoint(v, w, h), rtol=0, atol=1e-12)


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_loops_2d(fwd, adj):
    rng = np.random.default_rng(32)
    shape, m = (4, 6), 2
    u = rng.standard_normal(shape)
    w = rng.uniform(0, 1, (m,) + shape)
    h = rng.standard_normal((m,) + shape)
    assert np.allclose(fwd(u, w, h), _loops_2d(u, w, h), rtol=0, atol=1e-12)


def test_delta_responses_multiply_by_window_sum():
    # h_k = delta at lag 0: G_m u = (sum_k w_k) . u
    rng = np.random.default_rng(33)
    n, m = 24, 4
    w = rng.uniform(0, 1, (m, n))
    h = np.zeros((m, n))
    h[:, 0] = 1.0
    u = rng.standard_normal(n)
    for fwd, adj in FORMS:
        assert np.allclose(fwd(u, w, h), w.sum(0) * u, atol=1e-12)
        assert np.allclose(adj(u, w, h), w.sum(0) * u, atol=1e-12)


def test_delta_input_gives_windowed_shifted_responses():
    # u = delta_j: (G_m u)[i] = sum_k w_k[i] h_k[i - j]
    rng = np.random.default_rng(34)
    n, m, j = 20, 3, 7
    w = rng.uniform(0, 1, (m, n))
    h = rng.standard_normal((m, n))
    u = np.zeros(n)
    u[j] = 1.0
    want = sum(w[k] * np.roll(h[k], j) for k in range(m))
    for fwd, _ in FORMS:
        assert np.allclose(fwd(u, w, h), want, atol=1e-12)


def test_constant_windows_match_convolution_product_and_plain_convolution():
    rng = np.random.default_rng(35)
    n, m = 30, 3
    c = rng.uniform(0.5, 2.0, m)
    w = np.repeat(c[:, None], n, axis=1)
    h = rng.standard_normal((m, n))
    u = rng.standard_normal(n)
    assert np.allclose(ex.apply_pc_fft(u, w, h), ex.apply_fft(u, w, h), atol=1e-12)
    # one term, unit window: a plain circular convolution (numpy's FFT)
    want = np.real(np.fft.ifft(np.fft.fft(h[0]) * np.fft.fft(u)))
    assert np.allclose(ex.apply_pc_direct(u, np.ones((1, n)), h[:1]), want, atol=1e-12)


def test_adjoint_of_convolution_product_on_flipped_responses():
    # G_m(w, h) = H_m(w, h~)^*  (and G_m^* = H_m(w, h~))
    rng = np.random.default_rng(36)
    for shape in [(40,), (6, 10)]:
        m = 3
        w = rng.uniform(0, 1, (m,) + shape)
        h = rng.standard_normal((m,) + shape)
        u = rng.standard_normal(shape)
        ht = _flip(h)
        assert np.allclose(ex.apply_pc_fft(u, w, h), ex.adjoint_fft(u, w, ht), atol=1e-12)
        assert np.allclose(ex.adjoint_pc_fft(u, w, h), ex.apply_fft(u, w, ht), atol=1e-12)


@pytest.mark.parametrize("fwd,adj", FORMS)
def test_adjoint_identity(fwd, adj):
    rng = np.random.default_rng(37)
    n, m = 36, 4
    w = rng.uniform(0, 1, (m, n))
    h = rng.standard_normal((m, n))
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    assert abs(np.dot(fwd(u, w, h), v) - np.dot(u, adj(v, w, h))) < 1e-11


def test_sampled_outputs_match_full():
    rng = np.random.default_rng(38)
    for shape in [(50,), (7, 9)]:
        m = 3
        w = rng.uniform(0, 1, (m,) + shape)
        h = rng.standard_normal((m,) + shape)
        h[:, 2:-2] = 0.0 if len(shape) == 1 else h[:, 2:-2]
        u = rng.standard_normal(shape)
        idx = rng.choice(int(np.prod(shape)), 15, replace=False)
        yf = ex.apply_pc_fft(u, w, h).reshape(-1)[idx]
        xf = ex.adjoint_pc_fft(u, w, h).reshape(-1)[idx]
        assert np.allclose(ex.apply_pc_direct_at(u, w, h, idx), yf, atol=1e-12)
        assert np.allclose(ex.adjoint_pc_direct_at(u, w, h, idx), xf, atol=1e-12)


@pytest.mark.parametrize("shape", [(32,), (8, 12)])
def test_grad_spectra_finite_differences(shape):
    import scipy.fft as sfft
    rng = np.random.default_rng(39)
    m, nd = 3, len(shape)
    axes = tuple(range(-nd, 0))
    w = rng.uniform(0, 1, (m,) + shape)
    h = rng.standard_normal((m,) + shape)
    u = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    hs = sfft.rfftn(h, axes=axes)
    uh = sfft.rfftn(u, axes=axes)

    def loss(spec):
        y = sum(w[k] * sfft.irfftn(spec[k] * uh, s=shape, axes=axes) for k in range(m))
        return 0.5 * np.sum((y - f) ** 2)

    y = ex.apply_pc_fft(u, w, h)
    G = grads.grad_spectra_pc(u[None], (y - f)[None], w)
    eps = 1e-6
    last = shape[-1] // 2
    bins = [(0,) * nd, (0,) * (nd - 1) + (last,), (0,) * (nd - 1) + (1,)]
    if nd == 2:
        bins += [(3, 0), (5, last), (2, 4)]
    for k in range(m):
        for b in bins:
            for part in (1.0, 1j):
                hp, hm = hs.copy(), hs.copy()
                hp[(k,) + b] += eps * part
                hm[(k,) + b] -= eps * part
                fd = (loss(hp) - loss(hm)) / (2 * eps)
                an = G[(k,) + b].real if part == 1.0 else G[(k,) + b].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (k, b, part, fd, an)
