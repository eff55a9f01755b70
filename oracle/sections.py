"""Sectioned evaluation of the expansion as a function of per-section spectra
(TEST INFRASTRUCTURE: imported only by tests, the smoke check and the bench's
CPU baseline).

The compact-support lemma of section 3.5 (Lemma 3.2) evaluates term k of
eq. (1.4) only where it can be nonzero.  A section s of term k has, per axis,
a window box (origin o, extent p: every nonzero of w_k), a response lag box
(origin a, extent q: every nonzero of h_k) and a grid of M >= p + q - 1
samples.  On that grid:

* z_s holds (w_k . u) over the window box, placed at the grid origin, and
  zeros elsewhere;
* r_s holds h_k over the lag box, placed at the grid origin (lag a + i at
  index i), and zeros elsewhere;
* the circular convolution r_s * z_s on the grid equals the linear
  convolution of the two boxes (it spans p + q - 1 samples per axis, which
  fit in M), and it lands in the image at o + a.

So H_m u = sum_s place(r_s * z_s).  The section spectra S_s = rfft2(r_s) are
the operator's parameters here; ``apply_sections`` and its adjoint take them
as given (any complex values), ``grad_section_spectra`` is the gradient of a
loss with respect to them, each section being the one-term expansion
``irfft2(S_s . rfft2(z_s))`` of which only the first p + q - 1 samples per
axis are used.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import grads
from .expansion import workers

__all__ = ["circular_box", "section_geometry", "section_responses", "section_spectra", "apply_sections",
           "adjoint_sections", "grad_section_spectra"]


def circular_box(nonzero) -> tuple:
    """(origin, extent) of the shortest circular interval holding every True
    of a 1D mask; (0, 0) if there is none."""
    nz = np.flatnonzero(np.asarray(nonzero, bool))
    n = len(nonzero)
    if nz.size == 0:
        return 0, 0
    # the largest circular gap between consecutive nonzeros is left out
    gaps = np.diff(np.concatenate([nz, [nz[0] + n]]))
    g = int(np.argmax(gaps))
    start = int(nz[(g + 1) % nz.size])
    return start, n - int(gaps[g]) + 1


def _box2(a):
    o1, p1 = circular_box(np.any(a != 0, axis=1))
    o2, p2 = circular_box(np.any(a != 0, axis=0))
    return o1, p1, o2, p2


def section_geometry(w, h, length):
    """Sections of the terms with nonzero window and response: dicts with
    k, o1, p1, o2, p2, a1, q1, a2, q2, m1, m2; ``length(need, n)`` picks the
    grid size of an axis (at least ``need``)."""
    w = np.asarray(w)
    h = np.asarray(h)
    n1, n2 = w.shape[1:]
    out = []
    for k in range(w.shape[0]):
        o1, p1, o2, p2 = _box2(w[k])
        a1, q1, a2, q2 = _box2(h[k])
        if min(p1, p2, q1, q2) == 0:
            continue
        out.append(dict(k=k, o1=o1, p1=p1, o2=o2, p2=p2, a1=a1, q1=q1, a2=a2, q2=q2,
                        m1=length(p1 + q1 - 1, n1), m2=length(p2 + q2 - 1, n2)))
    return out


def _take(img, o1, o2, n1, n2):
    """The n1 x n2 block of the last two axes of img at (o1, o2), wrapped."""
    i = (o1 + np.arange(n1)) % img.shape[-2]
    j = (o2 + np.arange(n2)) % img.shape[-1]
    return img[..., i[:, None], j[None, :]]


def _add(img, blk, o1, o2):
    i = (o1 + np.arange(blk.shape[-2])) % img.shape[-2]
    j = (o2 + np.arange(blk.shape[-1])) % img.shape[-1]
    np.add.at(img, (Ellipsis, i[:, None], j[None, :]), blk)


def section_responses(h, secs):
    """r_s: h_k over its lag box, placed at the origin of the section grid."""
    out = []
    for s in secs:
        r = np.zeros((s["m1"], s["m2"]))
        r[:s["q1"], :s["q2"]] = _take(np.asarray(h[s["k"]], np.float64), s["a1"], s["a2"], s["q1"], s["q2"])
        out.append(r)
    return out


def section_spectra(h, secs):
    """S_s = rfft2(r_s)."""
    return [sfft.rfft2(r, workers=workers()) for r in section_responses(h, secs)]


def _z(u, w, s):
    """z_s for every signal of the batch u (B x N1 x N2)."""
    z = np.zeros((u.shape[0], s["m1"], s["m2"]))
    z[:, :s["p1"], :s["p2"]] = _take(np.asarray(w[s["k"]], np.float64)[None] * u, s["o1"], s["o2"], s["p1"], s["p2"])
    return z


def _ext(s):
    return min(s["p1"] + s["q1"] - 1, s["m1"]), min(s["p2"] + s["q2"] - 1, s["m2"])


def apply_sections(u, w, secs, spectra):
    """sum_s place(irfft2(S_s . rfft2(z_s))) over the first p + q - 1 samples
    per axis, for a batch u (B x N1 x N2) or one image."""
    u = np.asarray(u, np.float64)
    single = u.ndim == 2
    ub = u[None] if single else u
    y = np.zeros_like(ub)
    for s, S in zip(secs, spectra):
        ys = sfft.irfft2(S[None] * sfft.rfft2(_z(ub, w, s), workers=workers()), s=(s["m1"], s["m2"]),
                         workers=workers())
        e1, e2 = _ext(s)
        _add(y, ys[:, :e1, :e2], s["o1"] + s["a1"], s["o2"] + s["a2"])
    return y[0] if single else y


def _g(v, s):
    """The output box of section s read from v, on the section grid."""
    e1, e2 = _ext(s)
    g = np.zeros((v.shape[0], s["m1"], s["m2"]))
    g[:, :e1, :e2] = _take(v, s["o1"] + s["a1"], s["o2"] + s["a2"], e1, e2)
    return g


def adjoint_sections(v, w, secs, spectra):
    """The adjoint of apply_sections: sum_s w_k . place(the window box of
    irfft2(conj(S_s) . rfft2(g_s))), g_s the output box of v on the grid.
    Exact for section spectra of real responses (Hermitian-consistent)."""
    v = np.asarray(v, np.float64)
    single = v.ndim == 2
    vb = v[None] if single else v
    x = np.zeros_like(vb)
    for s, S in zip(secs, spectra):
        xs = sfft.irfft2(np.conj(S)[None] * sfft.rfft2(_g(vb, s), workers=workers()), s=(s["m1"], s["m2"]),
                         workers=workers())
        wb = _take(np.asarray(w[s["k"]], np.float64), s["o1"], s["o2"], s["p1"], s["p2"])
        _add(x, wb[None] * xs[:, :s["p1"], :s["p2"]], s["o1"], s["o2"])
    return x[0] if single else x


def grad_section_spectra(u, gy, w, secs):
    """dL/dS_s for y = apply_sections(u, ...) and gy = dL/dy, summed over the
    batch: the one-term expansion's spectra gradient on each section's grid
    (unit window, windowed input z_s, and the output box of gy, zero
    elsewhere on the grid: the rest of the section's output is unused)."""
    u = np.asarray(u, np.float64)
    gy = np.asarray(gy, np.float64)
    if u.ndim == 2:
        u, gy = u[None], gy[None]
    out = []
    for s in secs:
        one = np.ones((1, s["m1"], s["m2"]))
        out.append(grads.grad_spectra(_z(u, w, s), _g(gy, s), one)[0])
    return out
