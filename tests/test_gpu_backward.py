"""The differentiable form on the GPU: pc_apply_save / pc_backward on the
sectioned and full-grid 2D paths, the sections' spectra as parameters, and
the kept-or-recomputed windowed spectra (the plan's budget), against the FP64
oracle (the sectioned operator as a function of section spectra is pinned in
test_oracle_sections.py)."""
import os

import numpy as np
import pytest
import scipy.fft as sfft

import workloads as wl
from gpu_util import plan_args, rel_l2
from oracle import expansion as ex, grads
from oracle import sections as sc

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
    # tile windows with small PSFs: the plans section (one has a batch of 2)
    return [wl.small_2d(512, 512, 4, 4, 1, seed=61, kind="tile"),
            wl.small_2d(512, 768, 4, 4, 2, seed=62, kind="tile")]


def _secs(plan):
    out = []
    for s in plan.sections():
        out.append(dict(k=s["term"], o1=s["win_o1"], p1=s["win_p1"], o2=s["win_o2"], p2=s["win_p2"],
                        a1=s["lag_o1"], q1=s["lag_q1"], a2=s["lag_o2"], q2=s["lag_q2"], m1=s["m1"], m2=s["m2"],
                        off=s["spec_offset"]))
    return out


def _split(flat, secs):
    return [flat[s["off"]:s["off"] + s["m1"] * (s["m2"] // 2 + 1)].reshape(s["m1"], s["m2"] // 2 + 1) for s in secs]


@pytest.mark.parametrize("idx", range(2))
def test_sections_geometry_and_spectra(idx):
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    print(f"[gpu] sections of {p.name}", flush=True)
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True) as plan:
        assert plan.info()["path"] == 3
        secs = _secs(plan)
        spec = plan.get_spectra()
        torch.cuda.synchronize()
        got = spec.cpu().numpy()
    # every section covers its window and response supports with a grid of
    # at least p + q - 1 samples (the oracle's own boxes)
    ref = {s["k"]: s for s in sc.section_geometry(p.dense_windows(), p.h, lambda need, n: need)}
    assert sorted(s["k"] for s in secs) == sorted(ref)
    for s in secs:
        r = ref[s["k"]]
        for key in ("o1", "p1", "o2", "p2", "a1", "q1", "a2", "q2"):
            assert s[key] == r[key], (s, r)
        assert s["m1"] >= s["p1"] + s["q1"] - 1 and s["m2"] >= s["p2"] + s["q2"] - 1
    # the spectra layout: each section's real FFT of its shifted response
    for a, b in zip(_split(got, secs), sc.section_spectra(p.h, secs)):
        assert rel_l2(a, b) < 1e-6


@pytest.mark.parametrize("idx", range(2))
@pytest.mark.parametrize("mode", ["kept", "recomputed", "not_saved"])
def test_sectioned_backward_matches_oracle(idx, mode):
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    print(f"[gpu] sectioned backward {p.name} ({mode})", flush=True)
    rng = np.random.default_rng(70 + idx)
    gy = rng.standard_normal(p.u.shape).astype(np.float32)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True) as plan:
        if mode == "recomputed":
            plan.set_budget(0)
            assert plan.info()["keep_bytes"] == 0
        else:
            assert plan.info()["keep_bytes"] > 0
        secs = _secs(plan)
        y = plan.apply_save(u)
        gu, gs = plan.backward(u, torch.from_numpy(gy).cuda(), use_saved=mode != "not_saved")
        torch.cuda.synchronize()
        y, gu, gs = y.cpu().numpy(), gu.cpu().numpy(), gs.cpu().numpy()
    w = p.dense_windows()
    uu, g64 = p.u.astype(np.float64), gy.astype(np.float64)
    assert max(rel_l2(a, b) for a, b in zip(y, ex.apply_fft(uu, w, p.h.astype(np.float64)))) <= TOL
    assert max(rel_l2(a, b) for a, b in zip(gu, ex.adjoint_fft(g64, w, p.h.astype(np.float64)))) <= TOL
    ref = sc.grad_section_spectra(uu, g64, w, secs)
    err = max(rel_l2(a, b) for a, b in zip(_split(gs, secs), ref))
    print(f"{p.name} ({mode}): section spectra gradient rel {err:.2e}", flush=True)
    assert err <= TOL


def test_tuning_table_can_choose_recomputing():
    # a table entry "keep" = 0 makes a gradient plan recompute the windowed
    # spectra in the backward although they fit its budget; results unchanged
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[0]
    print(f"[gpu] keep = 0 through the tuning table {p.name}", flush=True)
    rng = np.random.default_rng(71)
    gy = rng.standard_normal(p.u.shape).astype(np.float32)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True) as plan:
        key = pcm.tune_key(plan.desc)
        assert plan.info()["keep_bytes"] > 0
    try:
        pcm.tune_set([(key, pcm.TUNE_KNOBS["keep"], 0, 0)])
        with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True) as plan:
            assert plan.info()["keep_bytes"] == 0
            secs = _secs(plan)
            plan.apply_save(u)
            gu, gs = plan.backward(u, torch.from_numpy(gy).cuda(), use_saved=True)
            torch.cuda.synchronize()
            gu, gs = gu.cpu().numpy(), gs.cpu().numpy()
    finally:
        path = pcm.tuning_table_path(pcm._device_arch())
        if path and os.path.exists(path):
            pcm.load_tuning(path)
        else:
            pcm.tune_set([])
    w = p.dense_windows()
    uu, g64 = p.u.astype(np.float64), gy.astype(np.float64)
    assert max(rel_l2(a, b) for a, b in zip(gu, ex.adjoint_fft(g64, w, p.h.astype(np.float64)))) <= TOL
    ref = sc.grad_section_spectra(uu, g64, w, secs)
    assert max(rel_l2(a, b) for a, b in zip(_split(gs, secs), ref)) <= TOL


def test_section_spectra_are_the_parameters():
    # replacing the sections' spectra (responses filling each grid) changes
    # the operator to the oracle's sectioned operator with those spectra
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[0]
    print(f"[gpu] section spectra as parameters {p.name}", flush=True)
    rng = np.random.default_rng(80)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True) as plan:
        secs = _secs(plan)
        S = [sfft.rfft2(rng.standard_normal((s["m1"], s["m2"])) * 1e-3) for s in secs]
        flat = np.concatenate([x.ravel() for x in S]).astype(np.complex64)
        plan.set_spectra(torch.from_numpy(flat).cuda())
        y = plan.apply(u).cpu().numpy()
        x = plan.apply_adjoint(u).cpu().numpy()
        back = plan.get_spectra().cpu().numpy()
    assert np.array_equal(back, flat)
    S32 = [a.astype(np.complex128) for a in _split(flat, secs)]
    w = p.dense_windows()
    uu = p.u.astype(np.float64)
    assert max(rel_l2(a, b) for a, b in zip(y, sc.apply_sections(uu, w, secs, S32))) <= TOL
    assert max(rel_l2(a, b) for a, b in zip(x, sc.adjoint_sections(uu, w, secs, S32))) <= TOL


@pytest.mark.parametrize("budget", [None, 0])
def test_full_grid_backward_matches_oracle(budget):
    import torch
    import paper_1604_04374_amd as pcm
    p = wl.small_2d(128, 192, 3, 2, 2, seed=63, kind="hat")
    print(f"[gpu] full-grid backward {p.name} (budget {budget})", flush=True)
    rng = np.random.default_rng(90)
    gy = rng.standard_normal(p.u.shape).astype(np.float32)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, gradients=True, full_grid=True) as plan:
        if budget is not None:
            plan.set_budget(budget)
        assert (plan.info()["keep_bytes"] > 0) == (budget is None)
        y = plan.apply_save(u)
        gu, gs = plan.backward(u, torch.from_numpy(gy).cuda(), use_saved=True)
        # a second backward without the saved state: the same numbers
        gu2, gs2 = plan.backward(u, torch.from_numpy(gy).cuda(), use_saved=False)
        torch.cuda.synchronize()
        y, gu, gs, gu2, gs2 = (t.cpu().numpy() for t in (y, gu, gs, gu2, gs2))
    w = p.dense_windows()
    h64, uu, g64 = p.h.astype(np.float64), p.u.astype(np.float64), gy.astype(np.float64)
    assert max(rel_l2(a, b) for a, b in zip(y, ex.apply_fft(uu, w, h64))) <= TOL
    assert max(rel_l2(a, b) for a, b in zip(gu, ex.adjoint_fft(g64, w, h64))) <= TOL
    assert rel_l2(gs, grads.grad_spectra(uu, g64, w)) <= TOL
    assert rel_l2(gu2, gu) <= 1e-6 and rel_l2(gs2, gs) <= 1e-6


def test_backward_argument_errors():
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[0]
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
        with pytest.raises(pcm.PCError) as ei:
            plan.backward(u, u)  # spectra gradient without PC_PLAN_GRADIENTS
        assert ei.value.status == 1
        gu, gs = plan.backward(u, u, want_spectra=False)
        torch.cuda.synchronize()
        ref = ex.adjoint_fft(p.u.astype(np.float64), p.dense_windows(), p.h.astype(np.float64))
        assert max(rel_l2(a, b) for a, b in zip(gu.cpu().numpy(), ref)) <= TOL
        with pytest.raises(pcm.PCError):
            plan.set_budget(-1)


@pytest.mark.parametrize("idx", range(2))
def test_sectioned_autograd_finite_differences(idx):
    import torch
    from paper_1604_04374_amd.autograd import ExpansionOperator, expansion
    p = _problems()[idx]
    print(f"[gpu] sectioned autograd {p.name}", flush=True)
    rng = np.random.default_rng(100 + idx)
    f = rng.standard_normal(p.u.shape).astype(np.float32)
    op = ExpansionOperator(plan_args(p), p.h, batch=p.batch)
    assert op.plan.info()["path"] == 3
    u = torch.from_numpy(p.u).cuda().requires_grad_(True)
    ft = torch.from_numpy(f).cuda()

    def loss_fn(uu, ss):
        r = expansion(uu, ss, op.plan) - ft
        return 0.5 * torch.sum(r.double() ** 2)

    loss = loss_fn(u, op.spec)
    loss.backward()
    gu = u.grad.detach().cpu().numpy()
    gs = op.spec.grad.detach().cpu().numpy()
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
@pytest.mark.parametrize("keep", [1, 0])
def test_c5_autograd_sectioned_full_size(keep):
    # the autograd workload at its stated size: 2048^2, 64 tile windows,
    # model PSFs, loss 0.5 ||H u - f||^2; gradients with respect to u and to
    # the 64 sections' spectra, against the oracle, with the windowed
    # spectra kept (keep = 1) or recomputed (keep = 0; the tuning table's
    # entry chooses it for the plan)
    import torch
    import paper_1604_04374_amd as pcm
    from paper_1604_04374_amd.autograd import ExpansionOperator
    p = wl.config_c5()
    w = p.dense_windows()
    print(f"[gpu] c5 autograd (sections, keep {keep}): oracle observation", flush=True)
    f = (ex.apply_fft(p.extra["u_true"].astype(np.float64), w, p.h.astype(np.float64))
         + 0.01 * p.extra["noise"]).astype(np.float32)
    op = ExpansionOperator(plan_args(p), p.extra["h_model"], batch=1)
    key = pcm.tune_key(op.plan.desc)
    del op
    try:
        pcm.tune_set([(key, pcm.TUNE_KNOBS["keep"], 0, keep)])
        op = ExpansionOperator(plan_args(p), p.extra["h_model"], batch=1)
    finally:
        path = pcm.tuning_table_path(pcm._device_arch())
        if path and os.path.exists(path):
            pcm.load_tuning(path)
        else:
            pcm.tune_set([])
    assert op.plan.info()["path"] == 3 and (op.plan.info()["keep_bytes"] > 0) == (keep == 1)
    secs = _secs(op.plan)
    u = torch.from_numpy(p.u).cuda().requires_grad_(True)
    y = op(u)
    loss = 0.5 * torch.sum((y - torch.from_numpy(f).cuda()) ** 2)
    loss.backward()
    gu = u.grad.cpu().numpy()
    gs = op.spec.grad.cpu().numpy()
    print("[gpu] c5 autograd (sections): oracle forward and gradients", flush=True)
    hm = p.extra["h_model"].astype(np.float64)
    uu = p.u.astype(np.float64)
    assert rel_l2(y.detach().cpu().numpy(), ex.apply_fft(uu, w, hm)) <= TOL
    r = y.detach().cpu().numpy().astype(np.float64) - f
    assert rel_l2(gu, ex.adjoint_fft(r, w, hm)) <= TOL
    ref = sc.grad_section_spectra(uu, r, w, secs)
    err = max(rel_l2(a, b) for a, b in zip(_split(gs, secs), ref))
    print(f"c5 sectioned gradient: worst section rel {err:.2e}", flush=True)
    assert err <= TOL
