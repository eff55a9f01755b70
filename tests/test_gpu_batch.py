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


@pytest.mark.parametrize("graph,persistent", [(True, False), (False, False), (True, True), (False, True)])
def test_batch_matches_oracle_and_single_plans(graph, persistent):
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(24)
    print(f"[gpu] batch of {len(plans)} (graph={graph}, persistent={persistent})", flush=True)
    b = pcm.Batch(plans, graph=graph, persistent=persistent)
    y = [t.clone() for t in b.apply(inputs)]
    x = [t.clone() for t in b.apply_adjoint(inputs)]
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


def test_new_tensors_on_every_call():
    # one batch (one captured graph per direction) applied to two sets of
    # tensors in turn, each against the oracle on its own inputs
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(10, seed=21)
    print("[gpu] batch on two sets of tensors", flush=True)
    rng = np.random.default_rng(22)
    second = [rng.uniform(0, 1, p.u.shape).astype(np.float32) for p in probs]
    inputs2 = [torch.from_numpy(v).cuda() for v in second]
    b = pcm.Batch(plans, graph=True)
    outs = []
    for rep in range(2):
        for ins in (inputs, inputs2):
            outs.append(([t.clone() for t in b.apply(ins)], [t.clone() for t in b.apply_adjoint(ins)]))
    torch.cuda.synchronize()
    for rep in range(2):
        for s, vals in enumerate((None, second)):
            y, x = outs[2 * rep + s]
            for i, p in enumerate(probs):
                ry, rx = oracle_fft(p) if vals is None else _oracle_on(p, vals[i])
                assert per_instance_rel(y[i].cpu().numpy(), ry) <= TOL, (rep, s, p.name)
                assert per_instance_rel(x[i].cpu().numpy(), rx) <= TOL, (rep, s, p.name)
    b.destroy()
    for pl in plans:
        pl.destroy()


def _oracle_on(p, u):
    from oracle import expansion as ex
    w = p.dense_windows()
    h = p.h.astype(np.float64)
    uu = u.astype(np.float64)
    return ex.apply_fft(uu, w, h), ex.adjoint_fft(uu, w, h)


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_are_identical_and_match_direct_launches(persistent):
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(16, seed=9)
    print(f"[gpu] batch graph replays (persistent={persistent})", flush=True)
    bg = pcm.Batch(plans, graph=True, persistent=persistent)
    first = [t.clone() for t in bg.apply(inputs)]
    firsta = [t.clone() for t in bg.apply_adjoint(inputs)]
    for rep in range(4):
        # eager work and synchronisation between replays
        z = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        ys = bg.apply(inputs)
        xs = bg.apply_adjoint(inputs)
        torch.cuda.synchronize()
        for a, b in zip(first, ys):
            assert torch.equal(a, b), rep
        for a, b in zip(firsta, xs):
            assert torch.equal(a, b), rep
        del z
    bg.destroy()
    bd = pcm.Batch(plans, graph=False, persistent=persistent)
    yd = bd.apply(inputs)
    xd = bd.apply_adjoint(inputs)
    torch.cuda.synchronize()
    for a, b in zip(first, yd):
        assert torch.equal(a, b)
    for a, b in zip(firsta, xd):
        assert torch.equal(a, b)
    bd.destroy()
    for pl in plans:
        pl.destroy()


@pytest.mark.slow
@pytest.mark.parametrize("persistent", [False, True])
def test_c4_full_size_batch(persistent):
    # the uneven-batch workload at its stated size: all 256 instances in one
    # batch, one graph launch per direction, every instance against the oracle
    import torch
    import paper_1604_04374_amd as pcm
    probs, plans, inputs = _setup(256, seed=4)
    print(f"[gpu] C4 full batch: {len(plans)} instances (persistent={persistent})", flush=True)
    b = pcm.Batch(plans, graph=True, persistent=persistent)
    y = b.apply(inputs)
    x = b.apply_adjoint(inputs)
    torch.cuda.synchronize()
    y = [t.cpu().numpy() for t in y]
    x = [t.cpu().numpy() for t in x]
    b.destroy()
    for pl in plans:
        pl.destroy()
    worst = 0.0
    for i, p in enumerate(probs):
        ry, rx = oracle_fft(p)
        ey, ex_ = per_instance_rel(y[i], ry), per_instance_rel(x[i], rx)
        worst = max(worst, ey, ex_)
        assert ey <= TOL and ex_ <= TOL, (p.name, ey, ex_)
    print(f"C4 full batch: worst rel-L2 {worst:.2e}", flush=True)


def test_batch_rejects_misuse():
    import ctypes
    import torch
    import paper_1604_04374_amd as pcm
    p = wl.config_c1()
    plan1d = pcm.Plan(p.w, p.h)
    with pytest.raises(pcm.PCError) as ei:
        pcm.Batch([plan1d])
    assert ei.value.status == 1
    plan1d.destroy()
    probs, plans, inputs = _setup(3, seed=30)
    # one plan listed twice: its instances would share the plan's workspace
    with pytest.raises(pcm.PCError) as ei:
        pcm.Batch([plans[0], plans[1], plans[0]])
    assert ei.value.status == 1
    b = pcm.Batch(plans)
    # a plan held by a live batch is not destroyed (and stays usable)
    lib = pcm.load_library()
    assert lib.pc_destroy(plans[1]._handle) == 1
    y = plans[1].apply(inputs[1])
    # overlapping outputs, an output overlapping an input, wrong counts
    with pytest.raises(pcm.PCError):
        b.apply(inputs, outputs=[inputs[0].clone(), inputs[1], torch.empty_like(inputs[2])])
    shared = torch.empty_like(inputs[0])
    if all(t.shape == inputs[0].shape for t in inputs):
        with pytest.raises(pcm.PCError):
            b.apply(inputs, outputs=[shared, shared, torch.empty_like(inputs[2])])
    with pytest.raises(ValueError):
        b.apply(inputs[:2])
    torch.cuda.synchronize()
    b.destroy()
    for pl in plans:
        pl.destroy()
    out = ctypes.c_void_p()
    assert lib.pc_batch_create(ctypes.byref(out), 0, None, 0, None) == 1
    assert lib.pc_batch_apply(None, None, None, None) == 1
    assert lib.pc_batch_destroy(None) == 1
    del y
