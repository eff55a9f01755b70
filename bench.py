#!/usr/bin/env python3
"""Throughput of the convolution-product expansion on one MI355X.

Workload (default): 64 real signals of N = 65536 samples sharing one
operator with m = 32 cubic B-spline windows and Gaussian impulse responses
(sigma(y) = 0.002 + 0.01 sin^2(pi y)), float32, seeded synthetic data.  One
step is the whole hot path over the batch: y = H_m u (pc_apply) and
x = H_m^* u (pc_apply_adjoint).  ``value`` counts the output samples of both
(2 x 64 x 65536 per step) per second, with the inputs already resident in
device memory.

The JSON line also carries
  * ``roofline``: the dominant kernel's algorithmic FP32 rate (flops per
    launch / average launch duration from HIP events recorded on the launch
    stream) against the chip's vector peak;
  * ``hbm``: algorithmic bytes per step over the step time against 8 TB/s;
  * ``cpu_baseline``: the FP64 oracle (FFT form) timed on the host cores on
    a bounded sample of the same workload, and its agreement with the GPU.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (256 CU x 2.4 GHz)
METRIC = "output samples/s for Hu and H*v at fixed m; achieved HBM GB/s fraction"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic work of the expansion (nominal FFT counts: 2.5 N log2 N flops
# per real transform of N points; complex MAC 8 flops per bin; one flop per
# windowed sample)
# ---------------------------------------------------------------------------

def algorithmic_counts_1d(n, m, batch, support_sum, inner_l, outer_r):
    nspec = n // 2 + 1
    fft = 2.5 * n * math.log2(n)
    per_sig_fwd = (m + 1) * fft + 8.0 * m * nspec + support_sum
    kernel_flops = {
        # forward: m transforms, MAC, windows, inner part of the inverse
        "fwd1d_large": batch * (m * fft + 8.0 * m * nspec + support_sum + 2.5 * n * math.log2(inner_l)),
        "combine1d": batch * (2.5 * n * math.log2(outer_r)),
        # adjoint: the forward transform of v, then m inverse transforms + MAC + windows
        "fold_fft": batch * fft,
        "adj1d_large": batch * (m * fft + 8.0 * m * nspec + support_sum),
        "ola1d": batch * float(n),
        "fwd1d_small": batch * per_sig_fwd,
        "adj1d_small": batch * per_sig_fwd,
    }
    bytes_dir = batch * n * 4 * 2 + m * nspec * 8 + support_sum * 4
    return {"flops_per_step": 2 * batch * per_sig_fwd, "bytes_per_step": 2 * bytes_dir,
            "kernel_flops": kernel_flops}


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = ["paper_1604_04374_amd/csrc/kern_1d.hip", "paper_1604_04374_amd/csrc/fft_engine.hpp"]


def read_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_src and m_b) or m_src.group(1) != source_digest(KERNEL_SOURCES):
        return None
    return float(m_b.group(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU work budget for the oracle baseline (0 disables it)")
    ap.add_argument("--no-trace", action="store_true", help="skip the per-kernel event pass")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the expansion shards with no communication across signals: see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1604_04374_amd as pcm
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    p = wl.config_c2()
    B, N, m = p.batch, p.shape[0], p.m
    log(f"[bench] workload {p.name}: building plan")
    plan = pcm.Plan(p.w, p.h, batch=B)
    info = plan.info()
    u = torch.from_numpy(p.u).to(dev)
    y = torch.empty_like(u)
    x = torch.empty_like(u)
    support_sum = int(np.count_nonzero(p.w))  # windows' nonzero samples (compact supports)
    counts = algorithmic_counts_1d(N, m, B, support_sum, info["fft_inner"], max(info["fft_outer"], 1))

    def step():
        plan.apply(u, out=y)
        plan.apply_adjoint(u, out=x)

    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    samples_per_step = 2 * B * N
    value = samples_per_step / (ms_per_step * 1e-3)

    roofline = None
    kernels = {}
    if not args.no_trace:
        log(f"[bench] per-kernel event pass ({args.steps} steps)")
        plan.set_tracing(True)
        plan.trace_reset()
        for _ in range(args.steps):
            step()
        kernels = plan.trace_stats()
        plan.set_tracing(False)
        dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
        name, st = dom
        flops = counts["kernel_flops"].get(name)
        if flops is not None and st["avg_ms"] > 0:
            achieved = flops / (st["avg_ms"] * 1e-3) / 1e12
            roofline = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                        "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "traffic": read_traffic(name, "c2"),
                        "avg_launch_ms": round(st["avg_ms"], 5),
                        "flops_per_launch": flops}
    hbm_gbps = counts["bytes_per_step"] / (ms_per_step * 1e-3) / 1e9

    cpu = None
    err = None
    if args.cpu_seconds > 0:
        from oracle import expansion as ex
        log("[bench] CPU oracle baseline")
        w64 = p.dense_windows()
        h64 = p.h.astype(np.float64)
        y_gpu = y.cpu().numpy()
        x_gpu = x.cpu().numpy()
        done = 0
        errs = []
        tc = 0.0
        while done < B and (tc < args.cpu_seconds or done == 0):
            uu = p.u[done:done + 1].astype(np.float64)
            c0 = time.perf_counter()
            ry = ex.apply_fft(uu, w64, h64)
            rx = ex.adjoint_fft(uu, w64, h64)
            tc += time.perf_counter() - c0
            errs.append(float(np.linalg.norm(y_gpu[done] - ry[0]) / np.linalg.norm(ry[0])))
            errs.append(float(np.linalg.norm(x_gpu[done] - rx[0]) / np.linalg.norm(rx[0])))
            done += 1
        cpu = {"value": round(2 * done * N / tc, 1), "unit": "samples/s", "cores": ex.workers(),
               "kind": "oracle",
               "sample": f"{done} of {B} signals, forward + adjoint, float64 FFT form (scipy.fft, "
                         f"{ex.workers()} workers), {tc:.1f} s"}
        err = max(errs)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1D batch 64 x N=65536, m=32 cubic B-spline windows, Gaussian h_k; "
                               "step = H_m u + H_m^* u",
                   "batch": B, "n": N, "m": m},
        "roofline": roofline,
        "hbm": {"alg_bytes_per_step": counts["bytes_per_step"], "achieved_GBps": round(hbm_gbps, 1),
                "peak_GBps": HBM_PEAK_GBPS, "frac": round(hbm_gbps / HBM_PEAK_GBPS, 4)},
        "alg_tflops": round(counts["flops_per_step"] / (ms_per_step * 1e-3) / 1e12, 3),
        "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in kernels.items()},
        "max_rel_l2_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    plan.destroy()


if __name__ == "__main__":
    main()
