"""The autotuner: measured choices of the per-length kernel variants.

For each workload it times, on the device, the alternatives of every knob
(include/pc.h PC_TUNE_*) that applies to one of its transform lengths, by
coordinate descent from the library's rule-based choices: one knob at a
time, a value is recorded only if it beats the current choices (the rules,
or the values recorded so far) by more than ``--margin``.  The choices are written to a JSON table keyed by
architecture, workload key, knob and length, which the binding loads at
start-up (``tuning/<arch>.json``).

    python -m paper_1604_04374_amd.tune --workloads c5 c5ad c3 c4 c2

Workloads (seeded synthetic inputs, as the benchmark's): c2 (1D batch of 64
signals of 65536 samples, m = 32), c3 (2D 1024^2, m = 16), c4 (256 uneven 2D
instances, one batch), c5 (2D 2048^2, m = 64 tiles, sectioned), c5ad (its
differentiable form: pc_apply_save + pc_backward).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import (Batch, Plan, TUNE_KNOBS, load_library, tune_batch_key, tune_key, tune_set, tuning_table_path,
               _device_arch)

KNOB_VALUES = {"cols_fwd_late": (0, 1), "cols_adj_prefetch": (0, 1), "rows_inv_pipe": (0, 1),
               "rows_fwd_small": (0, 1), "rows_inv_small": (0, 1)}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _problems(name):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as wl
    if name == "c2":
        return [wl.config_c2()]
    if name == "c3":
        return [wl.config_c3()]
    if name == "c4":
        return wl.config_c4()
    if name in ("c5", "c5ad"):
        return [wl.config_c5()]
    raise SystemExit(f"unknown workload {name}")


def _wins(p):
    return (p.w_rows, p.w_cols) if p.separable else p.w


class Workload:
    """Builds a workload's plans (and batch) and times its step."""

    def __init__(self, name):
        import torch
        self.name = name
        self.probs = _problems(name)
        self.inputs = [torch.from_numpy(p.u).cuda() for p in self.probs]
        self.plans = None
        self.batch = None
        if name == "c4":  # the batch's knobs are read at batch creation: the plans stay
            self.plans = [Plan(_wins(p), p.h, batch=p.batch, full_grid=True) for p in self.probs]

    def key(self):
        if self.name == "c4":
            return tune_batch_key(self.plans)
        self.build()
        return tune_key(self.plans[0].desc)

    def build(self):
        """(Re)create what reads the tuning table."""
        if self.name == "c4":
            if self.batch is not None:
                self.batch.destroy()
            self.batch = Batch(self.plans)
            return
        if self.plans:
            for pl in self.plans:
                pl.destroy()
        p = self.probs[0]
        self.plans = [Plan(_wins(p), p.h, batch=p.batch, gradients=self.name == "c5ad")]

    def lengths(self):
        """(column lengths, row lengths, 1D sizes) of the workload's transforms."""
        cols, rows, n1d = set(), set(), set()
        for pl in (self.plans or []):
            info = pl.info()
            if pl.desc.ndim == 1:
                n1d.add(int(pl.desc.n0))
            elif info["path"] == 3:
                for s in pl.sections():
                    cols.add(s["m1"])
                    rows.add(s["m2"])
            else:
                cols.add(int(pl.desc.n0))
                rows.add(int(pl.desc.n1))
        return sorted(cols), sorted(rows), sorted(n1d)

    def candidates(self):
        cols, rows, n1d = self.lengths()
        out = []
        for L in cols:
            out += [("cols_fwd_late", L, KNOB_VALUES["cols_fwd_late"]),
                    ("cols_adj_prefetch", L, KNOB_VALUES["cols_adj_prefetch"])]
        for L in rows:
            out += [(k, L, KNOB_VALUES[k]) for k in ("rows_fwd_small", "rows_inv_small", "rows_inv_pipe")]
        if self.name == "c4":
            out += [("batch_persistent", 0, (0, 1))]
        if self.name == "c5ad":
            out += [("keep", 0, (0, 1))]
        if self.name == "c3":
            pl = self.plans[0]
            nq = pl.desc.m_cols if pl.desc.w_format == 1 else pl.desc.m
            out += [("col_groups", int(pl.desc.n0), tuple(g for g in (1, 2, 4, 8, 16) if g <= nq))]
        for n in n1d:
            out += [("fourstep_l", n, tuple(l for l in (4096, 6144, 8192) if n % l == 0 and n // l in (2, 4, 8, 16)))]
        return out

    def step(self):
        import torch
        if self.name == "c4":
            self.batch.apply(self.inputs)
            self.batch.apply_adjoint(self.inputs)
        elif self.name == "c5ad":
            pl, u = self.plans[0], self.inputs[0]
            y = pl.apply_save(u)
            pl.backward(u, y, use_saved=True)
        else:
            pl, u = self.plans[0], self.inputs[0]
            pl.apply(u)
            pl.apply_adjoint(u)

    def time_ms(self, steps, reps=5):
        import torch
        for _ in range(3):
            self.step()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                self.step()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        return best

    def close(self):
        if self.batch is not None:
            self.batch.destroy()
        for pl in (self.plans or []):
            pl.destroy()


def tune_workload(name, others, steps, margin):
    """Coordinate descent over the workload's knobs; ``others``: entries of
    the other workloads (kept in the table while this one is timed)."""
    w = Workload(name)
    tune_set(others)
    key = w.key()
    chosen = {}  # (knob, length) -> value
    searched = []  # every knob timed: values and their step times

    def table():
        return others + [(key, TUNE_KNOBS[k], L, v) for (k, L), v in chosen.items()]

    w.build()
    best = w.time_ms(steps)
    _log(f"[tune] {name}: key {key:#018x}, rule-based step {best:.4f} ms")
    for knob, L, values in w.candidates():
        # the current choices (rules, or entries kept so far) are the
        # reference: an entry is kept only if one of the values beats it
        tune_set(table())
        w.build()
        ref = w.time_ms(steps)
        results = {}
        for v in values:
            tune_set(table() + [(key, TUNE_KNOBS[knob], L, v)])
            w.build()
            results[v] = w.time_ms(steps)
        v_best = min(results, key=results.get)
        searched.append(dict(workload=name, key=f"{key:#018x}", knob=knob, length=L, reference_ms=round(ref, 5),
                             ms={str(v): round(t, 5) for v, t in results.items()}))
        if results[v_best] < ref * (1.0 - margin):
            chosen[(knob, L)] = v_best
            best = results[v_best]
        _log(f"[tune] {name}: {knob}@{L}: current {ref:.4f}; " + ", ".join(f"{v}: {t:.4f}" for v, t in results.items())
             + (f" -> {chosen[(knob, L)]}" if (knob, L) in chosen else " -> rule kept"))
    tune_set(table())
    w.build()
    tuned = w.time_ms(steps)
    tune_set(others)
    w.build()
    rule = w.time_ms(steps)
    w.close()
    _log(f"[tune] {name}: rule-based {rule:.4f} ms, tuned {tuned:.4f} ms")
    entries = [dict(workload=name, key=f"{key:#018x}", knob=k, length=L, value=int(v))
               for (k, L), v in sorted(chosen.items())]
    return entries, {"rule_ms": round(rule, 5), "tuned_ms": round(tuned, 5), "searched": searched}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workloads", nargs="+", default=["c5", "c5ad", "c3", "c4", "c2"])
    ap.add_argument("--steps", type=int, default=20, help="steps per timing (best of 5)")
    ap.add_argument("--margin", type=float, default=0.01,
                    help="relative gain a knob change needs over the current choice")
    ap.add_argument("--out", default=None, help="table path (default: the package's tuning/<arch>.json)")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the tuner needs a GPU")
    load_library()
    arch = _device_arch()
    out = args.out or tuning_table_path(arch)
    entries, meas, searched = [], {}, []
    for name in args.workloads:
        others = [(int(e["key"], 16), TUNE_KNOBS[e["knob"]], e["length"], e["value"]) for e in entries]
        t0 = time.perf_counter()
        e, m = tune_workload(name, others, args.steps, args.margin)
        m["tuning_s"] = round(time.perf_counter() - t0, 1)
        entries += e
        searched += m.pop("searched")
        meas[name] = m
    os.makedirs(os.path.dirname(out), exist_ok=True)
    table = {"arch": arch, "device": torch.cuda.get_device_name(0),
             "method": "coordinate descent from the rule-based choices, best of 5 timings of "
                       f"{args.steps} steps per value, a change kept if it gains more than {args.margin:.0%}",
             "measurements": meas, "entries": entries, "searched": searched}
    with open(out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    tune_set([(int(e["key"], 16), TUNE_KNOBS[e["knob"]], e["length"], e["value"]) for e in entries])
    print(json.dumps({"table": out, "entries": len(entries), "measurements": meas}))


if __name__ == "__main__":
    main()
