"""GPU parity: the HIP library against the FP64 oracle, element by element.

Tolerance: relative L2 error <= 1e-5 per signal, forward and adjoint (FP32
complex arithmetic against float64 on the same float32 inputs).
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import (gpu_run, oracle_direct, oracle_fft, per_instance_rel, rel_l2,
                      sampled_direct, plan_args)

TOL = 1e-5

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()  # a missing library is a failure, not a skip


def _check(p, direct=False, samples=0):
    y, x = gpu_run(p)
    ry, rx = (oracle_direct(p) if direct else oracle_fft(p))
    ey, ex_ = per_instance_rel(y, ry), per_instance_rel(x, rx)
    print(f"{p.name}: fwd rel {ey:.2e} adj rel {ex_:.2e}", flush=True)
    assert ey <= TOL and ex_ <= TOL, (ey, ex_)
    if samples:
        es = sampled_direct(p, y, x, n_samples=samples)
        print(f"{p.name}: sampled direct rel {es:.2e}", flush=True)
        assert es <= TOL
    return y, x


# ---------------------------------------------------------------------------
# 1D, one workgroup per transform
# ---------------------------------------------------------------------------

def test_c1_forward_adjoint_vs_direct_sums():
    _check(wl.config_c1(), direct=True)


@pytest.mark.parametrize("n,m,deg,batch", [
    (64, 3, 1, 5), (96, 4, 3, 2), (128, 8, 1, 1), (192, 2, 1, 3), (256, 16, 3, 4),
    (384, 5, 3, 1), (512, 8, 1, 7), (768, 4, 1, 2), (1536, 6, 3, 3), (2048, 12, 3, 2),
    (3072, 3, 1, 1), (4096, 16, 3, 2), (6144, 6, 3, 3), (8192, 8, 3, 2), (256, 1, 1, 3),
    # enough pairs to fill the chip one pair per transform slot (the small
    # batches above split each pair's terms over a workgroup's slots)
    (256, 5, 1, 8200),
])
def test_1d_small_sizes(n, m, deg, batch):
    p = wl.small_1d(n, m, deg, batch, seed=100 + n, sigma_fn=lambda y: 0.01 + 0.03 * y)
    _check(p, direct=n <= 2048 and batch <= 64)


# ---------------------------------------------------------------------------
# 1D four-step (N = R * L)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,deg,batch", [
    (16384, 4, 3, 3), (12288, 5, 1, 2), (32768, 16, 3, 2), (24576, 8, 3, 1),
    (49152, 12, 1, 2), (98304, 16, 3, 1), (131072, 32, 3, 1),
    # C2's split (L = 4096, R = 16, two-chunk windows) with an odd batch: the
    # last pair's second signal is the plan's zero vector
    (65536, 32, 3, 3),
])
def test_1d_fourstep_sizes(n, m, deg, batch):
    p = wl.small_1d(n, m, deg, batch, seed=200 + m, sigma_fn=wl.gen.c2_sigma)
    _check(p, samples=64)


def test_1d_fourstep_wide_zero_and_wrapping_windows():
    # supports wider than the inner length (several adjoint chunks), an empty
    # window, and a window straddling index 0
    n = 16384
    rng = np.random.default_rng(7)
    w = np.zeros((4, n))
    w[0] = 0.5 + rng.uniform(0, 1, n)              # full support
    w[1, n - 3000:] = 1.0
    w[1, :5000] = 2.0                              # wraps around 0, 8000 wide
    w[3, 9000:9001] = 3.0                          # a single sample
    T = wl.tvir_gaussian(lambda y: 0.004 + 0.01 * y)
    h = wl.sample_h_1d(T, n, [0.1, 0.3, 0.5, 0.8])
    u = rng.standard_normal((3, n))
    p = wl.Problem(name="1d_special_windows", ndim=1, shape=(n,), m=4, batch=3,
                   u=u.astype(np.float32), h=h.astype(np.float32), w=w.astype(np.float32))
    _check(p, samples=32)


def test_c2_full_size():
    p = wl.config_c2()
    _check(p, samples=48)


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n1,n2,m1,m2,kind,batch", [
    (64, 64, 2, 2, "hat", 1), (64, 96, 3, 2, "hat", 2), (192, 128, 3, 2, "tile", 3),
    (128, 384, 2, 4, "hat", 1), (256, 256, 4, 4, "hat", 2), (512, 192, 4, 3, "tile", 1),
    # the longest transforms along each axis, and a single term
    (8192, 64, 2, 1, "hat", 1), (64, 8192, 1, 4, "tile", 2), (128, 128, 1, 1, "hat", 2),
])
def test_2d_separable(n1, n2, m1, m2, kind, batch):
    p = wl.small_2d(n1, n2, m1, m2, batch, seed=300 + n1 + n2, kind=kind)
    _check(p, direct=(n1 * n2 <= 64 * 96))


def test_2d_dense_windows():
    p = wl.small_2d(64, 128, 2, 3, 3, seed=41, kind="hat")
    w = p.dense_windows()
    rng = np.random.default_rng(5)
    w = w * rng.uniform(0.5, 1.5, w.shape)          # not separable any more
    p.w = w.astype(np.float32)
    p.w_rows = p.w_cols = None
    _check(p)


def test_c3_full_size():
    _check(wl.config_c3(), samples=48)


def test_c4_instances():
    probs = wl.config_c4(count=12, seed=4)
    for p in probs:
        _check(p, samples=16)


@pytest.mark.slow
def test_c5_full_size():
    _check(wl.config_c5(), samples=16)


# ---------------------------------------------------------------------------
# properties: adjoint identity, determinism, batch handling
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: wl.config_c1(),
    lambda: wl.small_1d(16384, 8, 3, 2, seed=9, sigma_fn=wl.gen.c2_sigma),
    lambda: wl.small_2d(128, 192, 2, 3, 1, seed=10),
])
def test_adjoint_identity_on_gpu(maker):
    import torch
    import paper_1604_04374_amd as pcm
    p = maker()
    rng = np.random.default_rng(11)
    u = torch.from_numpy(p.u).cuda()
    v = torch.from_numpy(rng.standard_normal(p.u.shape).astype(np.float32)).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
        hu = plan.apply(u).double()
        hv = plan.apply_adjoint(v).double()
        lhs = torch.sum(hu * v.double()).item()
        rhs = torch.sum(u.double() * hv).item()
        scale = hu.norm().item() * v.double().norm().item()
    assert abs(lhs - rhs) / scale < 1e-6


def test_repeat_is_bitwise_identical():
    import torch
    import paper_1604_04374_amd as pcm
    for p in (wl.small_1d(32768, 8, 3, 3, seed=12, sigma_fn=wl.gen.c2_sigma),
              wl.small_2d(128, 256, 2, 2, 2, seed=13), wl.config_c1()):
        u = torch.from_numpy(p.u).cuda()
        with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
            a, b = plan.apply(u), plan.apply(u)
            c, d = plan.apply_adjoint(u), plan.apply_adjoint(u)
            torch.cuda.synchronize()
            assert torch.equal(a, b) and torch.equal(c, d), p.name


def test_batch_smaller_than_capacity_and_zero():
    import ctypes
    import torch
    import paper_1604_04374_amd as pcm
    p = wl.small_1d(16384, 4, 3, 5, seed=14, sigma_fn=wl.gen.c2_sigma)
    ry, _ = oracle_fft(p)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=8) as plan:
        y3 = plan.apply(u[:3].contiguous())
        assert per_instance_rel(y3.cpu().numpy(), ry[:3]) <= TOL
        out = torch.full_like(u, 7.0)
        lib = pcm.load_library()
        st = lib.pc_apply(plan._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), 0, None)
        assert st == 0
        torch.cuda.synchronize()
        assert torch.all(out == 7.0)
        st = lib.pc_apply(plan._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), 9, None)
        assert st == 1
        st = lib.pc_apply(plan._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(u.data_ptr()), 1, None)
        assert st == 1


def test_destroyed_plan_is_rejected():
    import ctypes
    import paper_1604_04374_amd as pcm
    p = wl.config_c1()
    plan = pcm.Plan(plan_args(p), p.h, batch=1)
    h = ctypes.c_void_p(plan._handle.value)
    plan.destroy()
    lib = pcm.load_library()
    assert lib.pc_destroy(h) == 5
    assert lib.pc_apply(h, None, None, 1, None) == 5


@pytest.mark.parametrize("n,m,deg,expect", [
    # C2: cubic supports of 8192 = 2 x 4096 -> L = 4096, R = 16, one item per term
    (65536, 32, 3, (4096, 16, 32)),
    # hat supports of 2 N / m = 4915 <= 6144 -> L = 6144 (the only split), one item per term
    (12288, 5, 1, (6144, 2, 5)),
    # cubic supports of 24576 > 2 x 6144 -> long-support path, chunks of L samples
    (98304, 16, 3, (6144, 16, 16 * 4)),
])
def test_fourstep_split_choice(n, m, deg, expect):
    # the plan takes the shortest inner length whose windows fit in two
    # chunks (short-support kernels), else the long-support path
    import paper_1604_04374_amd as pcm
    p = wl.small_1d(n, m, deg, 1, seed=5, sigma_fn=wl.gen.c2_sigma)
    with pcm.Plan(plan_args(p), p.h, batch=1) as plan:
        info = plan.info()
    assert info["path"] == 1
    assert (info["fft_inner"], info["fft_outer"], info["n_items"]) == expect
