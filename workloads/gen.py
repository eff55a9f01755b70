"""Operator descriptions and seeded inputs (no expansion arithmetic here).

Discrete model shared by every consumer:

* 1D: the circle R/Z of the notation section, sampled at ``y_j = j/N``.  A
  lag index ``l`` stands for the signed offset ``lam(l) in [-1/2, 1/2)``
  (index 0 is zero lag, negative lags wrap to the end of the vector).
* 2D: an ``N1 x N2`` periodic image, row-major, ``N2`` contiguous; lags are
  signed pixel offsets per axis.
* The time-varying impulse response (TVIR) of the introduction is
  ``T(x, y) = K(x + y, y)``: ``T(., y)`` is the impulse response of the source
  point ``y``.  Impulse responses ``h_k`` are samples of ``T(., c_k)`` at a
  window centre ``c_k`` (the interpolation setting of section 4.4).
* Gaussians are unit-mass densities with standard deviation ``sigma``
  (Example 3.1); they are sampled, never cell-averaged or renormalised.
* B-spline windows follow the cardinal B-spline definition of the notation
  section: ``B_{0,m}`` is the indicator of width ``1/m`` and
  ``B_{a,m} = m B_{0,m} * B_{a-1,m}``, i.e. the centred cardinal B-spline of
  degree ``a`` on knots spaced ``1/m``; shifts ``k/m`` give a partition of
  unity on the circle.

Every random draw uses ``numpy.random.default_rng(seed)``.  GPU inputs are
float32; the oracle receives those same float32 values (upcast to float64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

__all__ = [
    "lag_unit", "lag_px", "grid_unit", "gaussian", "bspline_centered",
    "bspline_windows_1d", "tile_windows_1d", "tvir_gaussian",
    "sample_h_1d", "psf_aniso", "sample_h_2d", "Problem", "config_c1",
    "config_c2", "config_c3", "config_c4", "config_c5", "smooth_field",
    "small_1d", "small_2d", "example1_sigma", "example3_tvir",
    "expand_separable",
]


# ----------------------------------------------------------------------------
# grids and lags
# ----------------------------------------------------------------------------

def grid_unit(n: int) -> np.ndarray:
    """Sample positions ``y_j = j/n`` on [0, 1)."""
    return np.arange(n, dtype=np.float64) / n


def lag_px(n: int) -> np.ndarray:
    """Signed lag (in samples) of each index: ``((l + n//2) mod n) - n//2``."""
    l = np.arange(n)
    return (((l + n // 2) % n) - n // 2).astype(np.float64)


def lag_unit(n: int) -> np.ndarray:
    """Signed lag of each index on the unit circle, in [-1/2, 1/2)."""
    return lag_px(n) / n


def gaussian(x, sigma):
    """Unit-mass Gaussian density of standard deviation ``sigma`` (Example 3.1)."""
    x = np.asarray(x, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    return np.exp(-x * x / (2.0 * sigma * sigma)) / (math.sqrt(2.0 * math.pi) * sigma)


# ----------------------------------------------------------------------------
# windows
# ----------------------------------------------------------------------------

def bspline_centered(t, degree: int) -> np.ndarray:
    """Centred cardinal B-spline of the given degree, unit knot spacing.

    Closed forms of the recurrence ``B_a = B_0 * B_{a-1}`` (unit width):
    degree 0 is the indicator of [-1/2, 1/2) (half-open so that shifts tile
    the line), degree 1 the hat, degree 2 the quadratic, degree 3 the cubic
    (knot values 1/6, 2/3, 1/6).
    """
    t = np.asarray(t, dtype=np.float64)
    a = np.abs(t)
    if degree == 0:
        return ((t >= -0.5) & (t < 0.5)).astype(np.float64)
    if degree == 1:
        return np.maximum(1.0 - a, 0.0)
    if degree == 2:
        return np.where(a < 0.5, 0.75 - a * a,
                        np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    if degree == 3:
        return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                        np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))
    raise ValueError("degree must be 0, 1, 2 or 3")


def _wrap_unit(d):
    """Map a difference on the unit circle into [-1/2, 1/2)."""
    return d - np.floor(d + 0.5)


def bspline_windows_1d(n: int, m: int, degree: int, centres=None) -> np.ndarray:
    """``w_k[j] = B_{degree,m}(y_j - c_k)`` on the circle, ``c_k = k/m``.

    Returns an ``m x n`` float64 array.  For ``m >= degree + 1`` the rows sum
    to one at every sample (partition of unity).
    """
    y = grid_unit(n)
    c = np.arange(m) / m if centres is None else np.asarray(centres, np.float64)
    d = _wrap_unit(y[None, :] - c[:, None])
    return bspline_centered(d * m, degree)


def tile_windows_1d(n: int, m: int) -> np.ndarray:
    """Indicators of the ``m`` tiles ``[k n/m, (k+1) n/m)`` (Haar scaling span)."""
    if n % m:
        raise ValueError("n must be a multiple of m")
    w = np.zeros((m, n))
    s = n // m
    for k in range(m):
        w[k, k * s:(k + 1) * s] = 1.0
    return w


def expand_separable(w_rows: np.ndarray, w_cols: np.ndarray) -> np.ndarray:
    """Dense 2D windows ``w_{k1*m2+k2}[i1, i2] = a_{k1}[i1] * b_{k2}[i2]``."""
    m1, n1 = w_rows.shape
    m2, n2 = w_cols.shape
    out = w_rows[:, None, :, None] * w_cols[None, :, None, :]
    return out.reshape(m1 * m2, n1, n2)


# ----------------------------------------------------------------------------
# kernels / impulse responses
# ----------------------------------------------------------------------------

def tvir_gaussian(sigma_fn: Callable[[np.ndarray], np.ndarray]):
    """TVIR of Example 3.1: ``T(x, y) = g_{sigma(y)}(x)`` (sigma at the source)."""
    def T(x, y):
        return gaussian(x, sigma_fn(np.asarray(y, dtype=np.float64)))
    return T


def example1_sigma(y):
    """The smooth width field used for Example 3.1 in Figure 1."""
    return 0.08 + 0.02 * np.cos(2.0 * np.pi * np.asarray(y, np.float64))


def example3_tvir(sigma1: float = 0.05, sigma2: float = 0.1):
    """Example 3.3: two Gaussians switched by the indicator of |y| <= 1/4.

    ``y`` is read on the centred circle [-1/2, 1/2).
    """
    def T(x, y):
        yc = _wrap_unit(np.asarray(y, np.float64))
        ind = (np.abs(yc) <= 0.25).astype(np.float64)
        return gaussian(x, sigma1) * ind + gaussian(x, sigma2) * (1.0 - ind)
    return T


def sample_h_1d(T, n: int, centres) -> np.ndarray:
    """``h_k[l] = (1/n) T(lam(l), c_k)``: the quadrature weight times the
    impulse response of the source ``c_k``, in lag layout."""
    lam = lag_unit(n)
    c = np.asarray(centres, np.float64)
    return np.stack([T(lam, ck) for ck in c]) / n


def psf_aniso(n1: int, n2: int, sig_y: float, sig_x: float) -> np.ndarray:
    """Axis-aligned Gaussian PSF in lag layout, pixel units (sums to ~1)."""
    ly = lag_px(n1)
    lx = lag_px(n2)
    return gaussian(ly, sig_y)[:, None] * gaussian(lx, sig_x)[None, :]


def sample_h_2d(n1, n2, centres_px, sig_y_fn, sig_x_fn) -> np.ndarray:
    """PSF of each source pixel ``(p1, p2)`` in ``centres_px``."""
    hs = []
    for (p1, p2) in centres_px:
        hs.append(psf_aniso(n1, n2, float(sig_y_fn(p1, p2)), float(sig_x_fn(p1, p2))))
    return np.stack(hs)


def smooth_field(rng, n1, n2, modes=2):
    """Seeded random trigonometric polynomial (<= ``modes`` per axis), scaled
    so that its extreme absolute value on the pixel grid is 1."""
    coef = rng.standard_normal((modes + 1, modes + 1))
    phase = rng.uniform(0, 2 * np.pi, (modes + 1, modes + 1))
    coef[0, 0] = 0.0
    p1 = np.arange(n1)[:, None] / n1
    p2 = np.arange(n2)[None, :] / n2
    s = np.zeros((n1, n2))
    for a in range(modes + 1):
        for b in range(modes + 1):
            if coef[a, b] != 0.0:
                s += coef[a, b] * np.cos(2 * np.pi * (a * p1 + b * p2) + phase[a, b])
    return s / np.max(np.abs(s))


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """One operator plus a batch of inputs.

    ``u`` is ``batch x N`` (1D) or ``batch x N1 x N2`` (2D), float32.
    Windows are either dense (``w``: ``m x N`` / ``m x N1 x N2``) or a
    separable grid (``w_rows``: ``m1 x N1``, ``w_cols``: ``m2 x N2``, term
    ``k = k1*m2 + k2``).  ``h`` holds the impulse responses in lag layout,
    float32, same trailing shape as one signal.
    """
    name: str
    ndim: int
    shape: tuple
    m: int
    batch: int
    u: np.ndarray
    h: np.ndarray
    w: Optional[np.ndarray] = None
    w_rows: Optional[np.ndarray] = None
    w_cols: Optional[np.ndarray] = None
    T: Optional[Callable] = None          # 1D TVIR for the dense quadrature
    extra: dict = field(default_factory=dict)

    @property
    def separable(self) -> bool:
        return self.w_rows is not None

    def dense_windows(self) -> np.ndarray:
        """float64 dense windows (products of the float32 factors if separable)."""
        if self.w is not None:
            return self.w.astype(np.float64)
        return expand_separable(self.w_rows.astype(np.float64),
                                self.w_cols.astype(np.float64))

    @property
    def n_total(self) -> int:
        return int(np.prod(self.shape))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def small_1d(n=1024, m=8, degree=1, batch=1, seed=1, sigma_fn=None, dist="normal"):
    """1D problem: ``m`` B-spline windows of the given degree centred at
    ``k/m``, Gaussian TVIR with ``sigma`` at the source, ``h_k`` sampled at
    the window centres."""
    if sigma_fn is None:
        sigma_fn = lambda y: 0.01 + 0.02 * y  # noqa: E731
    rng = np.random.default_rng(seed)
    T = tvir_gaussian(sigma_fn)
    centres = np.arange(m) / m
    w = bspline_windows_1d(n, m, degree)
    h = sample_h_1d(T, n, centres)
    if dist == "normal":
        u = rng.standard_normal((batch, n))
    else:
        u = rng.uniform(0.0, 1.0, (batch, n))
    return Problem(name=f"1d_n{n}_m{m}_deg{degree}_b{batch}", ndim=1, shape=(n,),
                   m=m, batch=batch, u=_f32(u), h=_f32(h), w=_f32(w), T=T,
                   extra={"centres": centres, "degree": degree, "u64": u})


def config_c1():
    """1D, N=1024, m=8 hat windows on [0,1), sigma(y) = 0.01 + 0.02 y,
    u ~ N(0,1) (seed 1)."""
    p = small_1d(1024, 8, 1, 1, seed=1, sigma_fn=lambda y: 0.01 + 0.02 * y)
    p.name = "c1_1d_n1024_m8_hat"
    return p


def c2_sigma(y):
    return 0.002 + 0.01 * np.sin(np.pi * np.asarray(y, np.float64)) ** 2


def config_c2(batch=64, n=65536, m=32, seed=2):
    """1D batch of ``batch`` signals, N=65536, m=32 cubic B-spline windows,
    sigma(y) = 0.002 + 0.01 sin^2(pi y), u ~ N(0,1) float32 (seed 2)."""
    p = small_1d(n, m, 3, batch, seed=seed, sigma_fn=c2_sigma)
    p.name = f"c2_1d_b{batch}_n{n}_m{m}_cubic"
    return p


def _hat_grid_2d(n1, n2, m1, m2):
    return bspline_windows_1d(n1, m1, 1), bspline_windows_1d(n2, m2, 1)


def c3_sig_y(n1):
    return lambda p1, p2: 1.0 + 3.0 * p1 / n1


def c3_sig_x(n2):
    return lambda p1, p2: 1.0 + 3.0 * p2 / n2


def small_2d(n1=64, n2=64, m1=2, m2=2, batch=1, seed=3, kind="hat",
             sig_y_fn=None, sig_x_fn=None, dist="uniform"):
    """2D problem on a separable ``m1 x m2`` window grid (``hat`` B-splines
    centred on ``k/m`` per axis, or ``tile`` indicators) with an anisotropic
    Gaussian PSF evaluated at each window centre."""
    rng = np.random.default_rng(seed)
    if kind == "hat":
        a, b = _hat_grid_2d(n1, n2, m1, m2)
        c1 = [k * n1 / m1 for k in range(m1)]
        c2 = [k * n2 / m2 for k in range(m2)]
    elif kind == "tile":
        a, b = tile_windows_1d(n1, m1), tile_windows_1d(n2, m2)
        c1 = [(k + 0.5) * n1 / m1 for k in range(m1)]
        c2 = [(k + 0.5) * n2 / m2 for k in range(m2)]
    else:
        raise ValueError(kind)
    sy = sig_y_fn or c3_sig_y(n1)
    sx = sig_x_fn or c3_sig_x(n2)
    centres = [(p1, p2) for p1 in c1 for p2 in c2]
    h = sample_h_2d(n1, n2, centres, sy, sx)
    if dist == "uniform":
        u = rng.uniform(0.0, 1.0, (batch, n1, n2))
    else:
        u = rng.standard_normal((batch, n1, n2))
    return Problem(name=f"2d_{n1}x{n2}_m{m1}x{m2}_{kind}_b{batch}", ndim=2,
                   shape=(n1, n2), m=m1 * m2, batch=batch, u=_f32(u), h=_f32(h),
                   w_rows=_f32(a), w_cols=_f32(b),
                   extra={"centres_px": centres, "kind": kind})


def config_c3(n1=1024, n2=1024, seed=3):
    """2D 1024x1024, m=16 (4x4 separable hat grid), anisotropic Gaussian PSF
    with sigma_x, sigma_y growing linearly 1 -> 4 px across the image,
    u ~ U[0,1] (seed 3)."""
    p = small_2d(n1, n2, 4, 4, 1, seed=seed, kind="hat")
    p.name = f"c3_2d_{n1}x{n2}_m16_hat"
    return p


C4_SIDES = (128, 192, 256, 384, 512)
C4_M = (4, 9, 16)


def config_c4(count=256, seed=4, sides=C4_SIDES):
    """Uneven batch: ``count`` 2D instances with sides drawn independently from
    ``sides``, m from {4, 9, 16} (2x2 / 3x3 / 4x4 hat grids), PSF widths
    ``2.5 + 1.5 s(p)`` with ``s`` a seeded smooth random field in [-1, 1]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n1 = int(rng.choice(sides))
        n2 = int(rng.choice(sides))
        m = int(rng.choice(C4_M))
        g = int(round(math.sqrt(m)))
        sy = 2.5 + 1.5 * smooth_field(rng, n1, n2)
        sx = 2.5 + 1.5 * smooth_field(rng, n1, n2)
        sub_seed = int(rng.integers(0, 2**31 - 1))
        p = small_2d(n1, n2, g, g, 1, seed=sub_seed, kind="hat",
                     sig_y_fn=lambda p1, p2, s=sy: s[int(p1) % s.shape[0], int(p2) % s.shape[1]],
                     sig_x_fn=lambda p1, p2, s=sx: s[int(p1) % s.shape[0], int(p2) % s.shape[1]])
        p.name = f"c4_{i}_{n1}x{n2}_m{m}"
        out.append(p)
    return out


def config_c5(n=2048, tiles=8, seed=5, sigma_scale_model=1.25):
    """2D 2048x2048, m=64 tile windows (8x8 grid of 256x256 indicators, the
    span of the Haar scaling functions at level 3 per axis); PSFs of the C3
    family sampled at the tile centres.  ``h`` is the true operator; the
    model's PSFs use widths scaled by ``sigma_scale_model``.  Also returns
    ``u_true ~ U[0,1]`` and unit Gaussian noise (the observation
    ``f = H_true u_true + 0.01 noise`` needs the operator, so it is formed by
    the caller)."""
    rng = np.random.default_rng([seed, 1])
    p = small_2d(n, n, tiles, tiles, 1, seed=seed, kind="tile")
    sy = c3_sig_y(n)
    sx = c3_sig_x(n)
    h_model = sample_h_2d(n, n, p.extra["centres_px"],
                          lambda a, b: sigma_scale_model * sy(a, b),
                          lambda a, b: sigma_scale_model * sx(a, b))
    p.name = f"c5_2d_{n}x{n}_m{tiles * tiles}_tiles"
    p.extra["u_true"] = p.u.copy()
    p.extra["noise"] = _f32(rng.standard_normal((1, n, n)))
    p.extra["h_model"] = _f32(h_model)
    return p


def tvir_band_torch(n: int, sigma_fn, device, cutoff_sigmas: float = 15.0):
    """Rows of the TVIR ``T(lam, y) = g_{sigma(y)}(lam)`` (Example 3.1 form,
    unit-mass Gaussian of width ``sigma(y)`` at the source ``y = j/n``) for
    every lag within ``cutoff_sigmas`` times the largest width, generated on
    ``device`` in float64 and stored as float32 (beyond ~14.4 widths the
    float32 values are exact zeros).  Returns ``(rows x n tensor, lags)``
    with ``lags`` the rows' lag indices (lag layout)."""
    import torch
    y = np.arange(n) / n
    sig = np.asarray(sigma_fn(y), np.float64)
    cut = int(math.ceil(cutoff_sigmas * sig.max() * n))
    cut = min(cut, n // 2 - 1)
    lags = np.concatenate([np.arange(0, cut + 1), np.arange(n - cut, n)]).astype(np.int64)
    sig_t = torch.from_numpy(sig).to(device)
    out = torch.empty((lags.shape[0], n), dtype=torch.float32, device=device)
    lam_all = np.where(lags < n // 2, lags, lags - n) / n
    norm = 1.0 / (math.sqrt(2.0 * math.pi) * sig_t)
    for s0 in range(0, lags.shape[0], 1024):
        lam = torch.from_numpy(lam_all[s0:s0 + 1024]).to(device)[:, None]
        out[s0:s0 + 1024] = (torch.exp(-0.5 * (lam / sig_t[None, :]) ** 2) * norm[None, :]).float()
    return out, lags


def meyer_coefficients_random(n: int = 65536, n_mu: int = 32, n_lam: int = 4096, count: int = 20000,
                              seed: int = 6):
    """A seeded set of kept wavelet coefficients c_{lam, mu} for Meyer's
    representation: ``mu`` among the first ``n_mu`` basis vectors (the
    coarsest scaling functions), ``lam`` among the first ``n_lam`` (coarse
    scales), values N(0, 1) decaying like 1 / (1 + lam / 64)."""
    rng = np.random.default_rng(seed)
    lam = rng.integers(0, n_lam, count)
    mu = rng.integers(0, n_mu, count)
    c = rng.standard_normal(count) / (1.0 + lam / 64.0)
    return lam.astype(np.int64), mu.astype(np.int64), c.astype(np.float32)
