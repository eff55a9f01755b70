"""Periodic wavelet transforms and Meyer's operator representation (section
4.5) on the GPU against the FP64 oracle (`oracle.wavelets`, pinned in
test_oracle_wavelets.py).  Tolerance: rel-L2 <= 1e-5 (FP32 transforms of a
few taps per level; orthogonal, so nothing amplifies the rounding)."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import rel_l2
from oracle import dense, expansion as ex, wavelets as wv

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()


@pytest.mark.parametrize("N,n,levels,count", [(1, 64, 6, 3), (2, 256, 5, 4), (3, 1024, 7, 2), (4, 4096, 8, 5),
                                              (2, 8, 3, 2), (5, 512, 4, 1)])
def test_transform_rows_and_inverse(N, n, levels, count):
    import torch
    import paper_1604_04374_amd as pcm
    h = wv.daubechies(N)
    x = np.random.default_rng(N * 100 + n).standard_normal((count, n)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    c = pcm.wavelet_transform(xd, h, levels)
    assert rel_l2(c.cpu().numpy(), wv.dwt(x.astype(np.float64), h, levels)) <= TOL
    back = pcm.wavelet_transform(c, h, levels, inverse=True)
    assert rel_l2(back.cpu().numpy(), x) <= TOL


def test_transform_columns_and_2d_tvir_coefficients():
    import torch
    import paper_1604_04374_amd as pcm
    n, levels = 256, 5
    h = wv.daubechies(3)
    TT = dense.tvir_matrix_1d(wl.tvir_gaussian(lambda y: 0.02 + 0.01 * np.sin(2 * np.pi * y)), n)
    T32 = TT.astype(np.float32)
    d = torch.from_numpy(T32).cuda()
    rows = pcm.wavelet_transform(d, h, levels, axis=1)
    C = pcm.wavelet_transform(rows, h, levels, axis=0).cpu().numpy()
    assert rel_l2(C, wv.meyer_coefficients(T32.astype(np.float64), h, levels)) <= TOL


def _meyer_problem(n, levels, N, keep, seed):
    h = wv.daubechies(N)
    if n <= 4096:  # the largest coefficients of a TVIR
        TT = dense.tvir_matrix_1d(wl.tvir_gaussian(lambda y: 0.01 + 0.01 * np.sin(np.pi * y) ** 2), n)
        C = wv.meyer_coefficients(TT, h, levels)
        idx = np.argsort(np.abs(C).ravel())[::-1][:keep]
        lam, mu = np.unravel_index(idx, C.shape)
        return h, lam, mu, C[lam, mu].astype(np.float32)
    # random coefficients on the coarse scales (the first 64 basis vectors
    # in mu, the first 1024 in lambda), decaying with the index
    rng = np.random.default_rng(seed)
    lam = rng.integers(0, 1024, keep)
    mu = rng.integers(0, 64, keep)
    c = (rng.standard_normal(keep) / (1.0 + lam / 64.0)).astype(np.float32)
    return h, lam, mu, c


@pytest.mark.parametrize("n,levels,N,keep,batch", [(1024, 6, 2, 400, 3), (4096, 8, 3, 1500, 2),
                                                   (16384, 9, 4, 2000, 2)])
def test_meyer_plan_matches_oracle(n, levels, N, keep, batch):
    import torch
    import paper_1604_04374_amd as pcm
    print(f"[gpu] Meyer plan n={n} keep={keep}", flush=True)
    h, lam, mu, c = _meyer_problem(n, levels, N, keep, seed=n)
    plan = pcm.Plan.from_meyer(n, levels, h, lam, mu, c, batch=batch)
    mus, w, hk = wv.meyer_expansion(lam, mu, c.astype(np.float64), n, h, levels)
    assert plan.m == mus.shape[0]
    u = np.random.default_rng(n + 1).standard_normal((batch, n)).astype(np.float32)
    ud = torch.from_numpy(u).cuda()
    y = plan.apply(ud).cpu().numpy()
    x = plan.apply_adjoint(ud).cpu().numpy()
    plan.destroy()
    ry = ex.apply_fft(u.astype(np.float64), w, hk)
    rx = ex.adjoint_fft(u.astype(np.float64), w, hk)
    ey = max(rel_l2(a, b) for a, b in zip(y, ry))
    ea = max(rel_l2(a, b) for a, b in zip(x, rx))
    print(f"n={n}: {plan.m} terms, fwd rel {ey:.2e} adj rel {ea:.2e}", flush=True)
    assert ey <= TOL and ea <= TOL


def test_meyer_pipeline_on_device_coefficients():
    # the TVIR's coefficients computed by the device transforms, the largest
    # kept, the plan synthesised on the device; against the oracle's
    # expansion of the same kept set
    import torch
    import paper_1604_04374_amd as pcm
    n, levels, keep = 2048, 7, 800
    h = wv.daubechies(2)
    TT = dense.tvir_matrix_1d(wl.tvir_gaussian(lambda y: 0.01 + 0.01 * np.sin(np.pi * y) ** 2), n).astype(np.float32)
    d = torch.from_numpy(TT).cuda()
    C = pcm.wavelet_transform(pcm.wavelet_transform(d, h, levels, axis=1), h, levels, axis=0).cpu().numpy()
    idx = np.argsort(np.abs(C).ravel())[::-1][:keep]
    lam, mu = np.unravel_index(idx, C.shape)
    c = C[lam, mu]
    plan = pcm.Plan.from_meyer(n, levels, h, lam, mu, c, batch=1)
    u = np.random.default_rng(3).standard_normal(n).astype(np.float32)
    y = plan.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    plan.destroy()
    _, w, hk = wv.meyer_expansion(lam, mu, c.astype(np.float64), n, h, levels)
    assert rel_l2(y, ex.apply_fft(u.astype(np.float64), w, hk)) <= TOL
