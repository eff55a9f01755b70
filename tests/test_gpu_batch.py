"""Uneven batches (one graph launch for many 2D operators) against the
single-plan path and the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import oracle_fft, per_instance_rel, plan_args

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()


def _setup(count, seed=4):
    import torch
    import paper_1604_04374_amd as pcm
    probs = wl.config_c4(count=count, seed=seed)
    plans = [pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True) for p in probs]
    inputs = [torch.from_numpy(p.u).cuda() for p in probs]
    return probs, plans, inputs


@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_oracle_and_single_plans(graph):
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(24)
    print(f"[gpu] batch of {len(plans)} (graph={graph})", flush=True)
    b = pcm.Batch(plans, inputs, graph=graph)
    y = [t.clone() for t in b.apply()]
    x = [t.clone() for t in b.apply_adjoint()]
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        ry, rx = oracle_fft(p)
        assert per_instance_rel(y[i].cpu().numpy(), ry) <= TOL, p.name
        assert per_instance_rel(x[i].cpu().numpy(), rx) <= TOL, p.name
        ys = plans[i].apply(inputs[i])
        xs = plans[i].apply_adjoint(inputs[i])
        assert per_instance_rel(y[i].cpu().numpy(), ys.cpu().numpy()) <= 1e-6
        assert per_instance_rel(x[i].cpu().numpy(), xs.cpu().numpy()) <= 1e-6
    b.destroy()
    for pl in plans:
        pl.destroy()


def test_graph_replays_are_identical_and_match_direct_launches():
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(16, seed=9)
    print("[gpu] batch graph replays", flush=True)
    bg = pcm.Batch(plans, inputs, graph=True)
    first = [t.clone() for t in bg.apply()]
    firsta = [t.clone() for t in bg.apply_adjoint()]
    for rep in range(4):
        # eager work and synchronisation between replays
        z = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        ys = bg.apply()
        xs = bg.apply_adjoint()
        torch.cuda.synchronize()
        for a, b in zip(first, ys):
            assert torch.equal(a, b), rep
        for a, b in zip(firsta, xs):
            assert torch.equal(a, b), rep
        del z
    bg.destroy()
    bd = pcm.Batch(plans, inputs, graph=False)
    yd = bd.apply()
    xd = bd.apply_adjoint()
    torch.cuda.synchronize()
    for a, b in zip(first, yd):
        assert torch.equal(a, b)
    for a, b in zip(firsta, xd):
        assert torch.equal(a, b)
    bd.destroy()
    for pl in plans:
        pl.destroy()


def test_batch_rejects_1d_plans_and_bad_arguments():
    import ctypes
    import torch
    import paper_1604_04374_amd as pcm
    p = wl.config_c1()
    plan = pcm.Plan(p.w, p.h)
    u = torch.from_numpy(p.u).cuda()
    with pytest.raises(pcm.PCError):
        pcm.Batch([plan], [u])
    lib = pcm.load_library()
    out = ctypes.c_void_p()
    assert lib.pc_batch_create(ctypes.byref(out), 0, None, None, None, None, 0, None) == 1
    assert lib.pc_batch_apply(None, None) == 1
    assert lib.pc_batch_destroy(None) == 1
    plan.destroy()
