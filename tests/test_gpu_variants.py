"""GPU parity of the kernel variants the plans and batches choose per length,
forced through the tuning table (include/pc.h PC_TUNE_*).

Plan creation picks, per transform length, the forward column pass with
early or late spectrum loads, the adjoint column pass with or without the
next column's prefetch, the row-inverse pass with or without its pipelined
tile loads, and 16- or 4-row tiles for the row passes; a tuning table entry
for the workload overrides each rule.  Here every knob is forced on, then
off, for single plans and for a batch whose lengths take the other choice by
default, and the results are checked against the FP64 oracle (relative
L2 <= 1e-5); every entry of the committed tuning table is also forced on a
small workload of its length, with its value and with the other one.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from gpu_util import oracle_fft, per_instance_rel, plan_args

pytestmark = pytest.mark.gpu

TOL = 1e-5
SWITCHES = ("cols_fwd_late", "cols_adj_prefetch", "rows_inv_pipe", "rows_fwd_small", "rows_inv_small")
# (n1, n2, m1, m2, windows, batch): column lengths 256, 2048, 384, 192 and
# row lengths 256, 384, 2048, 768
CASES = [(256, 256, 4, 4, "hat", 2), (2048, 384, 2, 2, "hat", 1), (384, 2048, 2, 2, "tile", 1),
         (192, 768, 3, 2, "tile", 2)]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_04374_amd as pcm
    pcm.load_library()
    yield
    # back to the committed table for the tests that follow
    pcm.tune_set([])
    arch = pcm._device_arch()
    if arch and os.path.exists(pcm.tuning_table_path(arch)):
        pcm.load_tuning(pcm.tuning_table_path(arch))


def _force(key, lengths, values):
    import paper_1604_04374_amd as pcm
    pcm.tune_set([(key, pcm.TUNE_KNOBS[k], L, v) for k, v in values.items() for L in lengths])


def _run_plan(p, values):
    import torch
    import paper_1604_04374_amd as pcm
    lengths = set(p.shape)
    probe = pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True)
    key = pcm.tune_key(probe.desc)
    probe.destroy()
    _force(key, lengths, values)
    u = torch.from_numpy(p.u).cuda()
    with pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True) as plan:
        y = plan.apply(u).cpu().numpy()
        x = plan.apply_adjoint(u).cpu().numpy()
    pcm.tune_set([])
    return y, x


def _run_batch(probs, values):
    import torch
    import paper_1604_04374_amd as pcm
    plans = [pcm.Plan(plan_args(p), p.h, batch=p.batch, full_grid=True) for p in probs]
    key = pcm.tune_batch_key(plans)
    _force(key, set(L for p in probs for L in p.shape), values)
    inputs = [torch.from_numpy(p.u).cuda() for p in probs]
    b = pcm.Batch(plans)
    y = [t.cpu().numpy() for t in b.apply(inputs)]
    x = [t.cpu().numpy() for t in b.apply_adjoint(inputs)]
    b.destroy()
    for pl in plans:
        pl.destroy()
    pcm.tune_set([])
    return y, x


@pytest.mark.parametrize("forced", [1, 0])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}")
def test_forced_variants_match_oracle(forced, case):
    n1, n2, m1, m2, kind, batch = case
    p = wl.small_2d(n1, n2, m1, m2, batch, seed=700 + n1 + n2, kind=kind)
    print(f"{p.name}: every variant switch = {forced}", flush=True)
    y, x = _run_plan(p, {k: forced for k in SWITCHES})
    ry, rx = oracle_fft(p)
    ey, ex = per_instance_rel(y, ry), per_instance_rel(x, rx)
    print(f"{p.name}: fwd rel {ey:.2e} adj rel {ex:.2e}", flush=True)
    assert ey <= TOL and ex <= TOL, (ey, ex)


@pytest.mark.parametrize("forced", [1, 0])
def test_forced_variants_in_batches(forced):
    probs = [wl.small_2d(a, b, 2, 2, 1, seed=710 + a + b, kind="hat") for a, b in ((128, 192), (192, 256), (256, 128))]
    print(f"batch of {len(probs)}: every variant switch = {forced}", flush=True)
    y, x = _run_batch(probs, {k: forced for k in SWITCHES})
    for i, p in enumerate(probs):
        ry, rx = oracle_fft(p)
        assert per_instance_rel(y[i], ry) <= TOL and per_instance_rel(x[i], rx) <= TOL, p.name


def _table_entries():
    """The committed table's entries, then every other knob its tuner timed
    (with the value it found fastest)."""
    import paper_1604_04374_amd as pcm
    arch = pcm._device_arch()
    path = pcm.tuning_table_path(arch) if arch else None
    if not path or not os.path.exists(path):
        return []
    with open(path) as fh:
        table = json.load(fh)
    out = list(table["entries"])
    for srch in table.get("searched", []):
        best = min(srch["ms"], key=srch["ms"].get)
        out.append(dict(workload=srch["workload"], knob=srch["knob"], length=srch["length"], value=int(best)))
    return out


def test_every_tuning_table_entry_matches_oracle():
    # each entry of the committed table, with its value and the other
    # choices, on a small workload whose transforms have the entry's length
    entries = _table_entries()
    if not entries:
        pytest.skip("no tuning table for this device")
    seen = set()
    for e in entries:
        knob, L, v = e["knob"], int(e["length"]), int(e["value"])
        if (knob, L) in seen:
            continue
        seen.add((knob, L))
        print(f"table entry {e['workload']} {knob}@{L} = {v}", flush=True)
        if knob == "fourstep_l":
            p = wl.small_1d(L, 4, 3, 3, seed=720, sigma_fn=wl.gen.c2_sigma)
            for vv in sorted({v} | {l for l in (4096, 6144, 8192) if L % l == 0 and L // l in (2, 4, 8, 16)}):
                y, x = _run_plan(p, {knob: vv})
                ry, rx = oracle_fft(p)
                assert per_instance_rel(y, ry) <= TOL and per_instance_rel(x, rx) <= TOL, (knob, L, vv)
            continue
        if knob in ("batch_persistent", "sec_streams", "keep"):
            continue  # whole-launch choices, covered by the batch, section and backward tests
        if knob == "col_groups":
            p = wl.small_2d(L, 128, 2, 8, 1, seed=721, kind="hat")
            choices = sorted({v, 1, 2, 8})
        elif knob.startswith("cols"):
            p = wl.small_2d(L, 128, 2, 3, 2, seed=722, kind="hat")
            choices = [0, 1]
        else:
            p = wl.small_2d(128, L, 3, 2, 2, seed=723, kind="hat")
            choices = [0, 1]
        for vv in choices:
            y, x = _run_plan(p, {knob: vv})
            ry, rx = oracle_fft(p)
            assert per_instance_rel(y, ry) <= TOL and per_instance_rel(x, rx) <= TOL, (knob, L, vv)
