"""Pins of the sectioned-evaluation oracle (Lemma 3.2): exactness against the
plain expansion, the adjoint identity, the gradient by finite differences."""
import numpy as np
import pytest

from oracle import expansion as ex
from oracle import sections as sc

pytestmark = pytest.mark.filterwarnings("ignore")


def _problem(n1=48, n2=64, seed=3, radius=(5, 7)):
    """2D tiles (2 x 2 indicators) and responses with compact lag boxes
    (a Gaussian cut to |lag| <= radius, shifted off centre so the lag box
    wraps around the origin)."""
    rng = np.random.default_rng(seed)
    w = np.zeros((4, n1, n2))
    for k in range(4):
        i, j = divmod(k, 2)
        w[k, i * n1 // 2:(i + 1) * n1 // 2, j * n2 // 2:(j + 1) * n2 // 2] = 1.0
    h = np.zeros((4, n1, n2))
    for k in range(4):
        r1, r2 = radius
        d1, d2 = k - 1, 2 - k
        for a in range(-r1, r1 + 1):
            for b in range(-r2, r2 + 1):
                h[k, (a + d1) % n1, (b + d2) % n2] = np.exp(-(a * a + b * b) / (2.0 * (1.5 + k) ** 2))
    u = rng.standard_normal((2, n1, n2))
    return w, h, u


def _len_exact(need, n):
    return min(need, n)


def _len_pow2(need, n):
    m = 1
    while m < need:
        m *= 2
    return min(m, n)


def test_circular_box():
    assert sc.circular_box([0, 1, 1, 0, 0]) == (1, 2)
    assert sc.circular_box([1, 0, 0, 0, 1]) == (4, 2)      # wraps
    assert sc.circular_box([0, 0, 0]) == (0, 0)
    assert sc.circular_box([1, 1, 1, 1])[1] == 4
    assert sc.circular_box([1, 0, 1, 0, 0, 0]) == (0, 3)


@pytest.mark.parametrize("length", [_len_exact, _len_pow2])
def test_sections_equal_the_expansion(length):
    # Lemma 3.2: with grids of at least p + q - 1 samples per axis and the
    # sections' responses taken from h_k, the sum of sections is H_m u
    w, h, u = _problem()
    secs = sc.section_geometry(w, h, length)
    assert len(secs) == 4
    for s in secs:
        assert s["m1"] >= s["p1"] + s["q1"] - 1 and s["m2"] >= s["p2"] + s["q2"] - 1
    S = sc.section_spectra(h, secs)
    np.testing.assert_allclose(sc.apply_sections(u, w, secs, S), ex.apply_fft(u, w, h), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sc.adjoint_sections(u, w, secs, S), ex.adjoint_fft(u, w, h), rtol=1e-12, atol=1e-12)
    # and against the direct sums (one image)
    np.testing.assert_allclose(sc.apply_sections(u[0], w, secs, S), ex.apply_direct(u[0], w, h), rtol=1e-11,
                               atol=1e-11)


def test_short_grids_alias():
    # grids shorter than p + q - 1 wrap the linear convolution onto itself:
    # the lemma's bound is needed
    w, h, u = _problem()
    secs = sc.section_geometry(w, h, lambda need, n: min(need - 4, n))
    S = sc.section_spectra(h, secs)
    err = np.linalg.norm(sc.apply_sections(u, w, secs, S) - ex.apply_fft(u, w, h)) / np.linalg.norm(
        ex.apply_fft(u, w, h))
    assert err > 1e-3


def test_adjoint_identity_for_other_section_spectra():
    import scipy.fft as sfft
    w, h, u = _problem(seed=5)
    secs = sc.section_geometry(w, h, _len_pow2)
    rng = np.random.default_rng(6)
    # spectra of arbitrary real responses filling each grid
    S = [sfft.rfft2(rng.standard_normal((s["m1"], s["m2"]))) for s in secs]
    v = rng.standard_normal(u.shape)
    a = sc.apply_sections(u, w, secs, S)
    b = sc.adjoint_sections(v, w, secs, S)
    assert abs(np.sum(a * v) - np.sum(u * b)) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(v)


def test_grad_section_spectra_finite_differences():
    import scipy.fft as sfft
    w, h, u = _problem(n1=32, n2=40, seed=8, radius=(3, 4))
    secs = sc.section_geometry(w, h, _len_pow2)
    rng = np.random.default_rng(9)
    S = [sfft.rfft2(rng.standard_normal((s["m1"], s["m2"]))) for s in secs]
    f = rng.standard_normal(u.shape)

    def loss(Sx):
        r = sc.apply_sections(u, w, secs, Sx) - f
        return 0.5 * float(np.sum(r * r))

    gy = sc.apply_sections(u, w, secs, S) - f
    G = sc.grad_section_spectra(u, gy, w, secs)
    # the loss is quadratic in the spectra, so central differences are exact
    # up to rounding, which a larger step keeps small
    eps = 1e-3
    for si in (0, 3):
        m1, h2 = S[si].shape
        for b in [(0, 0), (0, h2 - 1), (1, 0), (3, 2), (m1 - 2, h2 - 1), (m1 // 2, 1)]:
            for part in (1.0, 1j):
                Sp = [x.copy() for x in S]
                Sm = [x.copy() for x in S]
                Sp[si][b] += eps * part
                Sm[si][b] -= eps * part
                fd = (loss(Sp) - loss(Sm)) / (2 * eps)
                an = G[si][b].real if part == 1.0 else G[si][b].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (si, b, part, fd, an)
