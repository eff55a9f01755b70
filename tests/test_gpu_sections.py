"""Sectioned 2D evaluation (compact supports, section 3.5 Lemma 3.2) against
the FP64 oracle, the full-grid plans and the direct sums.

Problems are built so that the plan takes the sectioned route (checked via
``info()["path"] == 3``): tile windows and narrow PSFs; hat windows whose
boxes wrap around the image edges; a grid that is sectioned along one axis
only; product-convolution plans; several images with partial batches.
Tolerance: relative L2 <= 1e-5 per image."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import per_instance_rel, plan_args, rel_l2
from oracle import expansion as ex

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()


def _narrow(a, b):
    return lambda p1, p2: a + b * (p1 + p2) / 1024.0


def _problems():
    return [
        wl.small_2d(256, 256, 4, 4, 2, seed=120, kind="tile", sig_y_fn=_narrow(1.0, 0.5), sig_x_fn=_narrow(1.2, 0.3)),
        wl.small_2d(512, 512, 8, 8, 1, seed=121, kind="hat", sig_y_fn=_narrow(1.0, 1.0), sig_x_fn=_narrow(1.5, 0.5)),
        wl.small_2d(128, 512, 1, 8, 3, seed=122, kind="tile", sig_y_fn=_narrow(1.0, 0.2), sig_x_fn=_narrow(1.0, 0.5)),
        wl.small_2d(384, 192, 6, 3, 1, seed=123, kind="tile", sig_y_fn=_narrow(0.8, 0.4), sig_x_fn=_narrow(1.0, 0.4)),
    ]


def _run(p, batch=None, **kw):
    import torch
    import paper_1604_04374_amd as pcm
    u = torch.from_numpy(p.u).cuda()
    if batch is not None:
        u = u[:batch].contiguous()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, **kw) as plan:
        info = plan.info()
        y = plan.apply(u).cpu().numpy()
        x = plan.apply_adjoint(u).cpu().numpy()
    return info, y, x


@pytest.mark.parametrize("idx", range(4))
def test_sectioned_matches_oracle_and_full_grid(idx):
    p = _problems()[idx]
    print(f"[gpu] sectioned {p.name}", flush=True)
    info, y, x = _run(p)
    print(f"{p.name}: path {info['path']} sections {info['n_items']} "
          f"{info['fft_inner']}x{info['fft_outer']}", flush=True)
    assert info["path"] == 3
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    ey = per_instance_rel(y, ex.apply_fft(u, w, h))
    ea = per_instance_rel(x, ex.adjoint_fft(u, w, h))
    print(f"{p.name}: fwd rel {ey:.2e} adj rel {ea:.2e}", flush=True)
    assert ey <= TOL and ea <= TOL
    finfo, yf, xf = _run(p, full_grid=True)
    assert finfo["path"] == 2
    assert per_instance_rel(y, yf) <= TOL and per_instance_rel(x, xf) <= TOL


@pytest.mark.parametrize("idx", [0, 1])
def test_sampled_direct_sums(idx):
    p = _problems()[idx]
    info, y, x = _run(p)
    assert info["path"] == 3
    rng = np.random.default_rng(130 + idx)
    w, h = p.dense_windows(), p.h.astype(np.float64)
    for b in range(p.batch):
        idxs = rng.choice(p.n_total, 256, replace=False)
        u = p.u[b].astype(np.float64)
        assert rel_l2(y[b].ravel()[idxs], ex.apply_direct_at(u, w, h, idxs)) <= TOL
        assert rel_l2(x[b].ravel()[idxs], ex.adjoint_direct_at(u, w, h, idxs)) <= TOL


@pytest.mark.parametrize("idx", [0, 2])
def test_partial_batch(idx):
    p = _problems()[idx]
    info, y, x = _run(p, batch=p.batch - 1)
    assert info["path"] == 3 and y.shape[0] == p.batch - 1
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u[:p.batch - 1].astype(np.float64)
    assert per_instance_rel(y, ex.apply_fft(u, w, h)) <= TOL
    assert per_instance_rel(x, ex.adjoint_fft(u, w, h)) <= TOL


@pytest.mark.parametrize("idx", [0, 1])
def test_product_convolution_sectioned(idx):
    p = _problems()[idx]
    print(f"[gpu] sectioned product-convolution {p.name}", flush=True)
    info, y, x = _run(p, product_convolution=True)
    assert info["path"] == 3
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    assert per_instance_rel(y, ex.apply_pc_fft(u, w, h)) <= TOL
    assert per_instance_rel(x, ex.adjoint_pc_fft(u, w, h)) <= TOL


def test_repeatable_bitwise_and_traced():
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[1]
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
        y1 = plan.apply(u).clone()
        x1 = plan.apply_adjoint(u).clone()
        plan.set_tracing(True)
        y2 = plan.apply(u)
        x2 = plan.apply_adjoint(u)
        stats = plan.trace_stats()
        plan.set_tracing(False)
        torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(x1, x2)
    # the row pass reads the input boxes in place: no separate gather
    assert "rows_fwd" in stats and "sec_scatter" in stats and "sec_gather" not in stats


def test_dense_windows_factored_or_kept_dense():
    # dense windows that are exactly a row factor times a column factor on
    # each box (tile indicators) are stored as the two factors; perturbed
    # ones keep a dense box; both against the oracle
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[0]
    w = p.dense_windows().astype(np.float32)
    rng = np.random.default_rng(130)
    w_bent = (w * (1.0 + 0.25 * rng.random(w.shape))).astype(np.float32)  # same supports, not rank one
    u = torch.from_numpy(p.u).cuda()
    nbytes = {}
    for name, ww in (("factored", w), ("dense", w_bent)):
        print(f"[gpu] sectioned {p.name}: {name} dense-format windows", flush=True)
        with pcm.Plan(ww, p.h, batch=p.batch) as plan:
            info = plan.info()
            assert info["path"] == 3
            nbytes[name] = info["window_bytes"]
            y = plan.apply(u).cpu().numpy()
            x = plan.apply_adjoint(u).cpu().numpy()
        h, uu = p.h.astype(np.float64), p.u.astype(np.float64)
        assert per_instance_rel(y, ex.apply_fft(uu, ww.astype(np.float64), h)) <= TOL
        assert per_instance_rel(x, ex.adjoint_fft(uu, ww.astype(np.float64), h)) <= TOL
    secs = None
    with pcm.Plan(w, p.h, batch=p.batch) as plan:
        secs = plan.sections()
    assert nbytes["factored"] == sum(4 * (s["m1"] + s["m2"]) for s in secs)
    assert nbytes["dense"] == sum(4 * s["m1"] * s["m2"] for s in secs)


@pytest.mark.parametrize("idx", [0, 1])
def test_two_launch_chains_match_one(idx):
    # the sections' two halves on two streams (the default) against one
    # chain on the call's stream (tuning entry PC_TUNE_SEC_STREAMS = 0): the
    # same kernels on the same data, so the outputs agree bit for bit
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[idx]
    u = torch.from_numpy(p.u).cuda()
    out = {}
    for v in (1, 0):
        with pcm.Plan(plan_args(p), p.h, batch=p.batch) as probe:
            key = pcm.tune_key(probe.desc)
        pcm.tune_set([(key, pcm.TUNE_KNOBS["sec_streams"], 0, v)])
        try:
            print(f"[gpu] sectioned {p.name}: sec_streams = {v}", flush=True)
            with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
                assert plan.info()["path"] == 3
                for _ in range(2):  # repeated calls reuse the fork and join events
                    y = plan.apply(u)
                    x = plan.apply_adjoint(u)
                out[v] = (y.cpu(), x.cpu())
        finally:
            pcm.tune_set([])
            arch = pcm._device_arch()
            if arch and __import__("os").path.exists(pcm.tuning_table_path(arch)):
                pcm.load_tuning(pcm.tuning_table_path(arch))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    w, h, uu = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    assert per_instance_rel(out[1][0].numpy(), ex.apply_fft(uu, w, h)) <= TOL
    assert per_instance_rel(out[1][1].numpy(), ex.adjoint_fft(uu, w, h)) <= TOL


def test_sectioned_plans_export_section_spectra():
    import torch
    import paper_1604_04374_amd as pcm
    p = _problems()[0]
    with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
        info = plan.info()
        assert info["path"] == 3
        # the parameters of a sectioned plan are its sections' spectra
        n = sum(s["m1"] * (s["m2"] // 2 + 1) for s in plan.sections())
        assert info["spectra_count"] == n and plan.get_spectra().shape == (n,)
        torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["graph", "direct", "persistent"])
def test_sectioned_plans_in_batches(mode):
    # sectioned plans (one with window boxes that partition the image, one
    # that does not, a product-convolution one) and a full-grid plan in one
    # batch; two calls with new tensors; every instance against the oracle
    # and against the plan's own calls
    import torch
    import paper_1604_04374_amd as pcm
    probs = _problems()
    specs = [(probs[0], False, False), (probs[1], False, False), (probs[3], True, False), (probs[2], False, True)]
    plans = [pcm.Plan(plan_args(p), p.h, batch=p.batch, product_convolution=pc, full_grid=fg) for p, pc, fg in specs]
    try:
        assert [pl.info()["path"] for pl in plans] == [3, 3, 3, 2]
        b = pcm.Batch(plans, graph=mode == "graph", persistent=mode == "persistent")
        try:
            for call in range(2):
                print(f"[gpu] batch of sectioned plans ({mode}), call {call}", flush=True)
                ins = [torch.from_numpy(p.u).cuda() * (1.0 + call) for p, _, _ in specs]
                ys = [t.clone() for t in b.apply(ins)]
                xs = [t.clone() for t in b.apply_adjoint(ins)]
                for k, ((p, pc, _), pl) in enumerate(zip(specs, plans)):
                    w, h = p.dense_windows(), p.h.astype(np.float64)
                    uu = p.u.astype(np.float64) * (1.0 + call)
                    ry = ex.apply_pc_fft(uu, w, h) if pc else ex.apply_fft(uu, w, h)
                    rx = ex.adjoint_pc_fft(uu, w, h) if pc else ex.adjoint_fft(uu, w, h)
                    assert per_instance_rel(ys[k].cpu().numpy(), ry) <= TOL, (mode, call, k)
                    assert per_instance_rel(xs[k].cpu().numpy(), rx) <= TOL, (mode, call, k)
                    y1, x1 = pl.apply(ins[k]), pl.apply_adjoint(ins[k])
                    assert rel_l2(ys[k].cpu().numpy(), y1.cpu().numpy()) <= 1e-6
                    assert rel_l2(xs[k].cpu().numpy(), x1.cpu().numpy()) <= 1e-6
        finally:
            b.destroy()
    finally:
        for pl in plans:
            pl.destroy()


@pytest.mark.slow
def test_c5_full_size():
    p = wl.config_c5()
    print(f"[gpu] sectioned {p.name}", flush=True)
    info, y, x = _run(p)
    print(f"{p.name}: path {info['path']} sections {info['n_items']} "
          f"{info['fft_inner']}x{info['fft_outer']}", flush=True)
    assert info["path"] == 3
    w, h, u = p.dense_windows(), p.h.astype(np.float64), p.u.astype(np.float64)
    assert per_instance_rel(y, ex.apply_fft(u, w, h)) <= TOL
    assert per_instance_rel(x, ex.adjoint_fft(u, w, h)) <= TOL
