"""The allocation-free wavelet transform (pc_wavelet_transform_noalloc)
against pc_wavelet_transform, through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DB2 = np.array([1 + 3 ** 0.5, 3 + 3 ** 0.5, 3 - 3 ** 0.5, 1 - 3 ** 0.5], np.float32) / np.float32(4 * 2 ** 0.5)
DB4 = np.array([0.2303778133088964, 0.7148465705529154, 0.6308807679298587, -0.0279837694168599,
                -0.1870348117190931, 0.0308413818355607, 0.0328830116668852, -0.0105974017850690], np.float32)


@pytest.fixture(scope="module")
def lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    return pcm.load_library()


def _call(lib, fn, x, out, lp, levels, inverse, count, n, stride, dist):
    import torch
    st = getattr(lib, fn)(1 if inverse else 0, n, levels, lp.shape[0], lp.ctypes.data_as(ctypes.c_void_p), count,
                          stride, dist, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.pc_last_error()


@pytest.mark.parametrize("order", ["large_then_small", "rows_then_columns"])
def test_noalloc_matches_allocating_call_twice(lib, order):
    import torch
    rng = np.random.default_rng(41)
    if order == "large_then_small":
        # (count, n, levels, inverse, stride/dist layout, filter): the second
        # call is smaller and leaves stale data of the first in the scratch
        cases = [(64, 8192, 6, False, "rows", DB4), (5, 512, 3, True, "rows", DB2)]
    else:
        cases = [(256, 1024, 4, True, "rows", DB2), (96, 256, 5, False, "cols", DB4)]
    for count, n, levels, inverse, layout, lp in cases:
        print(f"[gpu] noalloc {order}: count {count} n {n} levels {levels} inverse {inverse} {layout}", flush=True)
        if layout == "rows":
            x = torch.from_numpy(rng.standard_normal((count, n)).astype(np.float32)).cuda()
            stride, dist = 1, n
        else:
            x = torch.from_numpy(rng.standard_normal((n, count)).astype(np.float32)).cuda()
            stride, dist = count, 1
        ref = torch.empty_like(x)
        got = torch.full_like(x, float("nan"))
        _call(lib, "pc_wavelet_transform", x, ref, lp, levels, inverse, count, n, stride, dist)
        _call(lib, "pc_wavelet_transform_noalloc", x, got, lp, levels, inverse, count, n, stride, dist)
        torch.cuda.synchronize()
        # same kernels, same arithmetic: identical results
        assert torch.equal(got, ref), float((got - ref).abs().max())


def test_noalloc_rejects_requests_beyond_its_scratch(lib):
    import torch
    x = torch.zeros(1, device="cuda")
    lp = DB2
    # count * n = 2 * 4194304 > 4194304 samples: rejected before any launch
    st = lib.pc_wavelet_transform_noalloc(0, 1 << 22, 3, 4, lp.ctypes.data_as(ctypes.c_void_p), 2, 1, 1 << 22,
                                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + 4096),
                                          None)
    assert st == 1
    assert b"exceeds the fixed scratch" in lib.pc_last_error()
