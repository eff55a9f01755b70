"""Spectra as parameters and gradients on the GPU, against the FP64 oracle
(whose gradient formula is pinned by finite differences in test_oracle.py)
and against finite differences of the GPU loss itself."""
import numpy as np
import pytest
import scipy.fft as sfft

import workloads as wl
from gpu_util import plan_args, rel_l2
from oracle import expansion as ex, grads

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()


def _problems():
    return [
        wl.config_c1(),
        wl.small_1d(1536, 5, 3, 3, seed=21, sigma_fn=lambda y: 0.01 + 0.02 * y),
        wl.small_1d(16384, 6, 3, 3, seed=22, sigma_fn=wl.gen.c2_sigma),
        wl.small_1d(24576, 5, 1, 2, seed=23, sigma_fn=wl.gen.c2_sigma),
        wl.small_2d(64, 96, 2, 3, 3, seed=24, kind="hat"),
        wl.small_2d(128, 128, 4, 4, 1, seed=25, kind="tile"),
    ]


def _spec64(p):
    nd = p.ndim
    return sfft.rfftn(p.h.astype(np.float64), axes=tuple(range(-nd, 0)))


@pytest.mark.parametrize("idx", range(6))
def test_get_spectra_is_the_real_fft_of_h(idx):
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    print(f"[gpu] get_spectra {p.name}", flush=True)
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True) as plan:
        s = plan.get_spectra()
        torch.cuda.synchronize()
        got = s.cpu().numpy()
    assert rel_l2(got, _spec64(p)) < 1e-6


@pytest.mark.parametrize("idx", range(6))
def test_set_spectra_replaces_the_operator(idx):
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    print(f"[gpu] set_spectra {p.name}", flush=True)
    rng = np.random.default_rng(30 + idx)
    # a second operator: impulse responses of different widths
    h2 = np.roll(p.h, 3, axis=-1) * rng.uniform(0.5, 1.5, (p.m,) + (1,) * p.ndim)
    spec2 = sfft.rfftn(h2.astype(np.float64), axes=tuple(range(-p.ndim, 0)))
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True) as plan:
        plan.set_spectra(torch.from_numpy(spec2.astype(np.complex64)).cuda())
        y = plan.apply(u).cpu().numpy()
        x = plan.apply_adjoint(u).cpu().numpy()
    spec2_32 = spec2.astype(np.complex64).astype(np.complex128)
    w = p.dense_windows()
    ry = ex.apply_fft(p.u.astype(np.float64), w, None, h_spec=spec2_32)
    rx = ex.adjoint_fft(p.u.astype(np.float64), w, None, h_spec=spec2_32)
    assert max(rel_l2(a, b) for a, b in zip(y, ry)) <= TOL
    assert max(rel_l2(a, b) for a, b in zip(x, rx)) <= TOL


@pytest.mark.parametrize("idx", range(6))
def test_grad_spectra_matches_oracle(idx):
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    print(f"[gpu] grad_spectra {p.name}", flush=True)
    rng = np.random.default_rng(40 + idx)
    g = rng.standard_normal(p.u.shape).astype(np.float32)
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True, full_grid=True) as plan:
        gs = plan.grad_spectra(torch.from_numpy(p.u).cuda(), torch.from_numpy(g).cuda())
        torch.cuda.synchronize()
        got = gs.cpu().numpy()
    ref = grads.grad_spectra(p.u, g, p.dense_windows())
    err = rel_l2(got, ref)
    print(f"{p.name}: grad spectra rel {err:.2e}", flush=True)
    assert err <= TOL


def test_grad_spectra_requires_the_flag():
    import torch
    import paper_1604_04374_amd as pcm
    p = wl.config_c1()
    with pcm.Plan(plan_args(p), p.h) as plan:
        u = torch.from_numpy(p.u).cuda()
        with pytest.raises(pcm.PCError) as ei:
            plan.grad_spectra(u, u)
        assert ei.value.status == 1


@pytest.mark.parametrize("idx", [0, 2, 4])
def test_autograd_matches_oracle_and_finite_differences(idx):
    import torch
    from paper_1604_04374_amd.autograd import ExpansionOperator
    p = _problems()[idx]
    print(f"[gpu] autograd {p.name}", flush=True)
    rng = np.random.default_rng(50 + idx)
    f = rng.standard_normal(p.u.shape).astype(np.float32)
    op = ExpansionOperator(plan_args(p), p.h, batch=p.batch, full_grid=True)
    u = torch.from_numpy(p.u).cuda().requires_grad_(True)
    ft = torch.from_numpy(f).cuda()

    def loss_fn(uu, ss):
        from paper_1604_04374_amd.autograd import expansion
        r = expansion(uu, ss, op.plan) - ft
        return 0.5 * torch.sum(r.double() ** 2)

    loss = loss_fn(u, op.spec)
    loss.backward()
    gu = u.grad.detach().cpu().numpy()
    gs = op.spec.grad.detach().cpu().numpy()
    # oracle, with the float32 spectra the plan holds: forward, then the
    # backward on the GPU's own residual
    w = p.dense_windows()
    spec = op.spec.detach().cpu().numpy().astype(np.complex128)
    with torch.no_grad():
        from paper_1604_04374_amd.autograd import expansion
        y_gpu = expansion(u, op.spec, op.plan).cpu().numpy()
    y_ref = ex.apply_fft(p.u.astype(np.float64), w, None, h_spec=spec)
    assert max(rel_l2(a, b) for a, b in zip(y_gpu, y_ref)) <= TOL
    r = y_gpu.astype(np.float64) - f
    ref_gu = ex.adjoint_fft(r, w, None, h_spec=spec)
    ref_gs = grads.grad_spectra(p.u, r, w)
    assert rel_l2(gu, ref_gu) <= TOL
    assert rel_l2(gs, ref_gs) <= TOL
    # directional finite differences of the GPU loss: the loss is exactly
    # quadratic in u and in the spectra, so central differences are exact for
    # any step; a step of the size of the data keeps the difference far above
    # the rounding of the loss itself
    with torch.no_grad():
        du = torch.from_numpy(rng.standard_normal(p.u.shape).astype(np.float32)).cuda()
        # along the computed gradient (plus a seeded random part): the
        # loss change then stands well above the float32 rounding of the loss
        gdir = torch.from_numpy(gs).cuda()
        noise = torch.from_numpy((rng.standard_normal(gs.shape) + 1j * rng.standard_normal(gs.shape))
                                 .astype(np.complex64)).cuda()
        ds = (gdir / gdir.abs().mean() + 0.5 * noise) * op.spec.abs().mean()
        eps = 0.5
        fd_u = (loss_fn(u + eps * du, op.spec) - loss_fn(u - eps * du, op.spec)).item() / (2 * eps)
        an_u = float(np.sum(gu.astype(np.float64) * du.cpu().numpy()))
        assert abs(fd_u - an_u) <= 1e-3 * max(abs(an_u), 1e-12) + 1e-6
        sp = op.spec.detach()
        fd_s = (loss_fn(u, sp + eps * ds) - loss_fn(u, sp - eps * ds)).item() / (2 * eps)
        dsn = ds.cpu().numpy()
        an_s = float(np.sum(gs.real * dsn.real + gs.imag * dsn.imag))
        assert abs(fd_s - an_s) <= 1e-3 * max(abs(an_s), 1e-12) + 1e-6


@pytest.mark.slow
def test_c5_autograd_full_grid():
    # the 2048^2, 64-term operator kept on the full grid: spectra of h_k
    import torch
    from paper_1604_04374_amd.autograd import ExpansionOperator
    p = wl.config_c5()
    w = p.dense_windows()
    print("[gpu] c5 autograd (full grid): oracle observation", flush=True)
    f = (ex.apply_fft(p.extra["u_true"].astype(np.float64), w, p.h.astype(np.float64))
         + 0.01 * p.extra["noise"]).astype(np.float32)
    op = ExpansionOperator(plan_args(p), p.extra["h_model"], batch=1, full_grid=True)
    assert op.plan.info()["path"] == 2
    u = torch.from_numpy(p.u).cuda().requires_grad_(True)
    y = op(u)
    loss = 0.5 * torch.sum((y - torch.from_numpy(f).cuda()) ** 2)
    loss.backward()
    gu = u.grad.cpu().numpy()
    gs = op.spec.grad.cpu().numpy()
    spec = op.spec.detach().cpu().numpy().astype(np.complex128)
    print("[gpu] c5 autograd (full grid): oracle forward and gradients", flush=True)
    y_ref = ex.apply_fft(p.u.astype(np.float64), w, None, h_spec=spec)
    assert rel_l2(y.detach().cpu().numpy(), y_ref) <= TOL
    # the backward pass is checked on the upstream gradient the GPU produced:
    # the residual y - f is far smaller than y, so its rounding is amplified
    # and would otherwise dominate the comparison
    r = y.detach().cpu().numpy().astype(np.float64) - f
    assert rel_l2(gu, ex.adjoint_fft(r, w, None, h_spec=spec)) <= TOL
    assert rel_l2(gs, grads.grad_spectra(p.u, r, w)) <= TOL
