"""GPU parity of the kernel variants the plans choose per length.

Plan creation picks, per transform length, the forward column pass with
early or late spectrum loads, the adjoint column pass with or without the
next column's prefetch, and the row-inverse pass with or without its
pipelined tile loads (from the runtime's occupancy figures).  The default
tests run each variant only at the lengths where it is chosen; here the
tuning overrides (read at every plan creation) force every one of them on,
then off, for 2D plans whose lengths take the other choice by default, and
the results are checked against the FP64 oracle (relative L2 <= 1e-5, as in
the other parity tests).
"""
import os

import pytest

import workloads as wl
from gpu_util import gpu_run, oracle_fft, per_instance_rel

pytestmark = pytest.mark.gpu

TOL = 1e-5
OVERRIDES = ("PC_COLS_FWD_LATE", "PC_COLS_ADJ_PREFETCH", "PC_ROWS_INV_PIPE")
# (n1, n2, m1, m2, windows, batch): column lengths 256, 2048, 384, 192 and
# row lengths 256, 384, 2048 (small row tiles), 768
CASES = [(256, 256, 4, 4, "hat", 2), (2048, 384, 2, 2, "hat", 1), (384, 2048, 2, 2, "tile", 1),
         (192, 768, 3, 2, "tile", 2)]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()


@pytest.fixture
def forced_env(request):
    saved = {v: os.environ.get(v) for v in OVERRIDES}
    for v in OVERRIDES:
        os.environ[v] = request.param
    yield request.param
    for v, old in saved.items():
        if old is None:
            os.environ.pop(v, None)
        else:
            os.environ[v] = old


@pytest.mark.parametrize("forced_env", ["1", "0"], indirect=True)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}")
def test_forced_variants_match_oracle(forced_env, case):
    n1, n2, m1, m2, kind, batch = case
    p = wl.small_2d(n1, n2, m1, m2, batch, seed=700 + n1 + n2, kind=kind)
    print(f"{p.name}: variant overrides = {forced_env}", flush=True)
    y, x = gpu_run(p)
    ry, rx = oracle_fft(p)
    ey, ex = per_instance_rel(y, ry), per_instance_rel(x, rx)
    print(f"{p.name}: fwd rel {ey:.2e} adj rel {ex:.2e}", flush=True)
    assert ey <= TOL and ex <= TOL, (ey, ex)
