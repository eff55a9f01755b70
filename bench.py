#!/usr/bin/env python3
"""Throughput of the convolution-product expansion on one MI355X.

Workload (default, ``--workload c5``): one 2048 x 2048 float32 image and the
operator with m = 64 terms of 8 x 8 tile windows (256 x 256 indicators) and
anisotropic Gaussian PSFs sampled at the tile centres, seeded synthetic data,
evaluated section by section (the compact-support lemma, Lemma 3.2).  One
step is the whole hot path: y = H_m u (pc_apply) and x = H_m^* u
(pc_apply_adjoint).  ``value`` counts the output samples of both
(2 x 2048 x 2048 per step) per second, with the inputs already resident in
device memory.  The other workloads (``--workload``) are the 1D and uneven
batch configurations and the autograd step.

The JSON line also carries
  * ``roofline``: for the 2D workloads the whole step, HBM-bound: the
    method's algorithmic bytes per step (inputs read, outputs written, the
    plan's spectra and windows, each once per direction) over the step time
    from HIP events recorded on the launch stream around the timed region,
    against 8 TB/s; ``traffic`` is the counter-measured bytes of the step's
    kernels (committed summary under profiles/, when it matches the current
    kernel sources).  For the 1D batch (VALU-bound) the dominant kernel's
    algorithmic FP32 rate against the vector peak;
  * ``kernels``: every kernel family's average launch time (HIP events on
    the launch stream), its bytes as a separate pass (intermediate planes
    included) and its share of the step;
  * ``cpu_baseline``: the FP64 oracle (FFT form) timed on the host cores on
    a bounded sample of the same workload, and its agreement with the GPU;
  * ``cold_ms_per_step``: the median of steps timed one by one, each after a
    1 GiB write that leaves none of the step's data in L2 or the Infinity
    Cache (``ms_per_step`` is the warm rate of back-to-back steps);
  * ``hbm.copy_GBps``: a plain device copy's measured rate, with the HBM
    fractions also quoted against it (``frac_of_copy``).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

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
# per real transform of N points, 5 N log2 N per complex one; complex MAC 8
# flops per bin; one flop per windowed sample).  Bytes: the signals read and
# written, the m half-spectra and the windows' nonzero samples, per direction.
# ---------------------------------------------------------------------------

def _lg(x):
    return math.log2(x) if x > 1 else 0.0


def algorithmic_counts(p, info):
    """Per-step (forward + adjoint) flops and bytes, and per-kernel-family
    flops and bytes for one plan of workload ``p`` (batch ``p.batch``)."""
    B, m = p.batch, p.m
    ntot = p.n_total
    # nonzero window samples over all terms (the compacted windows); a
    # separable grid's term (k1, k2) has nnz(a_k1) nnz(b_k2) of them
    support_sum = int(np.count_nonzero(p.dense_windows())) if p.ndim == 1 else (
        int(np.count_nonzero(p.w_rows)) * int(np.count_nonzero(p.w_cols))
        if p.separable else int(np.count_nonzero(p.w)))
    if p.ndim == 1:
        n = p.shape[0]
        nspec = n // 2 + 1
        fft = 2.5 * n * _lg(n)
        per_sig = (m + 1) * fft + 8.0 * m * nspec + support_sum
        L, R = info["fft_inner"], max(info["fft_outer"], 1)
        kf = {
            "fwd1d_large": B * (m * fft + 8.0 * m * nspec + support_sum + 2.5 * n * _lg(L)),
            "combine1d": B * 2.5 * n * _lg(R),
            "fold_fft": B * fft,
            "adj1d_large": B * (m * fft + 8.0 * m * nspec + support_sum),
            "ola1d": B * float(n),
            "fwd1d_small": B * per_sig,
            "adj1d_small": B * per_sig,
        }
        spec_bytes = m * nspec * 8
        kb = {"fwd1d_large": B * n * 4 + spec_bytes + support_sum * 4, "adj1d_large": spec_bytes + support_sum * 4,
              "fwd1d_small": B * n * 8 + spec_bytes + support_sum * 4,
              "adj1d_small": B * n * 8 + spec_bytes + support_sum * 4}
    elif info["path"] == 3:
        # sectioned (compact supports): every section is a one-term operator
        # on fft_inner x fft_outer samples (the sizes are equal across
        # sections for the workloads here); the spectra are those of the
        # sections
        s_n, m1s, m2s = info["n_items"], info["fft_inner"], info["fft_outer"]
        h2s = m2s // 2 + 1
        rowfft = 2.5 * m1s * m2s * _lg(m2s)
        colfft = 5.0 * m1s * h2s * _lg(m1s)
        spec_bytes = s_n * m1s * h2s * 8
        per_sig = s_n * (2 * rowfft + 2 * colfft + 8.0 * m1s * h2s) + support_sum
        img_s, pl_s = m1s * m2s * 4, m1s * h2s * 8    # one section image / half-spectrum plane, bytes
        kf = {"rows_fwd": B * s_n * 2 * rowfft, "rows_inv": B * s_n * 2 * rowfft,
              "cols_fwd": B * s_n * (2 * colfft + 8.0 * m1s * h2s),
              "cols_adj": B * s_n * (2 * colfft + 8.0 * m1s * h2s)}  # one term: the column pass transforms V itself
        # per step (forward + adjoint); each family runs once or twice per step
        kb = {"cols_fwd": B * s_n * 2 * pl_s + spec_bytes, "cols_adj": B * s_n * 2 * pl_s + spec_bytes,
              "rows_fwd": 2 * B * s_n * (img_s + pl_s), "rows_inv": 2 * B * s_n * (img_s + pl_s),
              "sec_scatter": 2 * B * (s_n * img_s + ntot * 4)}
        bytes_dir = B * ntot * 4 * 2 + spec_bytes + support_sum * 4
        return {"flops_per_step": 2 * B * per_sig, "bytes_per_step": 2 * bytes_dir, "kernel_flops": kf,
                "kernel_bytes": kb}
    else:
        n1, n2 = p.shape
        h2 = n2 // 2 + 1
        nq = m if not p.separable else p.w_cols.shape[0]
        m1 = 1 if not p.separable else p.w_rows.shape[0]
        per_sig = (m + 1) * 2.5 * ntot * _lg(ntot) + 8.0 * m * n1 * h2 + support_sum
        rowfft = 2.5 * n1 * n2 * _lg(n2)
        colfft = 5.0 * n1 * h2 * _lg(n1)
        spec_bytes = m * n1 * h2 * 8
        kf = {"rows_fwd": B * (nq + 1) * rowfft, "rows_inv": B * (nq + 1) * rowfft,
              "cols_fwd": B * ((m + 1) * colfft + 8.0 * m * n1 * h2),
              "cols_adj": B * ((m + 1) * colfft + 8.0 * m * n1 * h2)}
        plane = n1 * h2 * 8
        # per step (forward + adjoint): the row passes move the image and the
        # planes of the row-transformed windowed copies (nq forward, 1 adjoint
        # and the reverse on the way out); the column passes move those planes
        # and the spectra
        kb = {"cols_fwd": B * (nq + 1) * plane + spec_bytes, "cols_adj": B * (nq + 1) * plane + spec_bytes,
              "cols_fft": 2 * B * plane, "cols_sum": B * 2 * plane,
              "rows_fwd": B * (2 * ntot * 4 + (nq + 1) * plane), "rows_inv": B * (2 * ntot * 4 + (nq + 1) * plane)}
    bytes_dir = B * ntot * 4 * 2 + m * (ntot // p.shape[-1]) * (p.shape[-1] // 2 + 1) * 8 + support_sum * 4
    return {"flops_per_step": 2 * B * per_sig, "bytes_per_step": 2 * bytes_dir, "kernel_flops": kf,
            "kernel_bytes": kb}


WORKLOADS = {
    "c1": "1D N=1024, m=8 hat windows, Gaussian h_k (sigma 0.01 + 0.02 y), batch 1",
    "c2": "1D batch 64 x N=65536, m=32 cubic B-spline windows, Gaussian h_k; step = H_m u + H_m^* u",
    "c3": "2D 1024x1024, m=16 (4x4 separable hat grid), anisotropic Gaussian PSF 1->4 px, batch 1",
    "c4": "256 uneven 2D instances, sides in {128,192,256,384,512}, m in {4,9,16}, one plan each",
    "c5": "2D 2048x2048, m=64 (8x8 tile windows), Gaussian PSFs, batch 1",
    "c5ad": "2D 2048x2048, m=64 tiles, sectioned: autograd step of 0.5||H_m u - f||^2 (forward, du and the "
            "sections' spectra gradient from one backward call), against the plain forward + adjoint",
    "c2pc": "1D batch 64 x N=65536, m=32 cubic B-spline windows, Gaussian h_k, product-convolution form "
            "G_m u = sum_k w_k . (h_k * u); step = G_m u + G_m^* u",
    "c5full": "2D 2048x2048, m=64 (8x8 tile windows), Gaussian PSFs, batch 1, evaluated on the full grid "
              "(no sections)",
    "c2proj": "construction: L2 projection (section 4.2) of the C2 TVIR band (all lags within 15 widths, "
              "65536 positions) onto the 32 cubic B-spline windows, on the device",
    "c2meyer": "Meyer representation (section 4.5): 1D batch 64 x N=65536, 20000 kept coefficients, 4-tap "
               "Daubechies wavelets at 11 levels, windows = the 32 coarsest scaling functions, responses "
               "synthesised on the device; step = H_m u + H_m^* u",
}
MEYER_LEVELS = 11
MFMA_FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
PRODUCT_CONVOLUTION = {"c2pc"}
# batched instances must be full-grid plans; c5full measures C5 without sections
FULL_GRID = {"c4", "c5full"}


def make_problems(name):
    import workloads as wl
    if name == "c1":
        return [wl.config_c1()]
    if name in ("c2", "c2pc"):
        return [wl.config_c2()]
    if name == "c2meyer":
        # the windows (for the algorithmic counts) are the library's own
        # synthesis of the unit coefficient vectors; the CPU leg rebuilds
        # windows and responses with the oracle
        import torch
        import paper_1604_04374_amd as pcm
        p = wl.config_c2()
        n = p.shape[0]
        lam, mu, c = wl.gen.meyer_coefficients_random(n)
        lp = np.array([1 + 3 ** 0.5, 3 + 3 ** 0.5, 3 - 3 ** 0.5, 1 - 3 ** 0.5]) / (4 * 2 ** 0.5)  # 4-tap Daubechies
        mus = np.unique(mu)
        e = torch.zeros((mus.shape[0], n), dtype=torch.float32, device="cuda")
        e[torch.arange(mus.shape[0]), torch.from_numpy(mus).cuda()] = 1.0
        p.w = pcm.wavelet_transform(e, lp, MEYER_LEVELS, inverse=True).cpu().numpy()
        p.h = None
        p.m = int(mus.shape[0])
        p.extra["meyer"] = (lam, mu, c)
        p.extra["lowpass"] = lp
        p.name = "c2meyer"
        return [p]
    if name == "c3":
        return [wl.config_c3()]
    if name == "c4":
        return wl.config_c4()
    if name in ("c5", "c5ad", "c5full"):
        return [wl.config_c5()]
    raise SystemExit(f"unknown workload {name}")


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {1: ["paper_1604_04374_amd/csrc/kern_1d.hip", "paper_1604_04374_amd/csrc/fft_engine.hpp"],
                  2: ["paper_1604_04374_amd/csrc/kern_2d.hip", "paper_1604_04374_amd/csrc/kern_sec.hip",
                      "paper_1604_04374_amd/csrc/fft_engine.hpp"]}


def read_traffic(kernel, workload, ndim):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_(?:launch|step):\s*([0-9.eE+]+)", text)
    if not (m_src and m_b) or m_src.group(1) != source_digest(KERNEL_SOURCES[ndim]):
        return None
    return float(m_b.group(1))


def measure_copy_gbps(torch, dev, mib=512, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    a plain torch copy of ``mib`` MiB, best of ``reps``: the attainable HBM
    rate the fractions are also quoted against."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU work budget for the oracle baseline (0 disables it)")
    ap.add_argument("--no-trace", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs of c4 (single-plan calls) and c5ad (plain step)")
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS),
                    help="c5 (default) is the reported configuration; the others are extra reports")
    ap.add_argument("--cold-steps", type=int, default=10,
                    help="extra steps timed one by one after a 1 GiB write that evicts L2 and the "
                         "Infinity Cache (reported as cold_ms_per_step; 0 disables)")
    ap.add_argument("--persistent", action="store_true",
                    help="c4: one persistent launch per pass (PC_BATCH_PERSISTENT)")
    ap.add_argument("--no-tuning", action="store_true",
                    help="clear the tuning table: every variant from the library's rules")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes 5 times (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(signals shard across GPUs with no communication; terms and image bands need one sum or halo exchange per step)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1604_04374_amd as pcm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    pcm.load_library()
    if args.no_tuning:
        pcm.tune_set([])

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 5}))
        return

    if args.workload == "c2proj":
        return bench_construct(args, torch, pcm, dev)

    probs = make_problems(args.workload)
    log(f"[bench] workload {args.workload}: {len(probs)} plan(s)")
    jobs = []
    counts = {"flops_per_step": 0.0, "bytes_per_step": 0.0, "kernel_flops": {}, "kernel_bytes": {}}
    for p in probs:
        wins = (p.w_rows, p.w_cols) if p.separable else p.w
        if args.workload == "c2meyer":
            t0 = time.perf_counter()
            lam, mu, c = p.extra["meyer"]
            plan = pcm.Plan.from_meyer(p.shape[0], MEYER_LEVELS, p.extra["lowpass"], lam, mu, c, batch=p.batch)
            torch.cuda.synchronize()
            log(f"[bench] Meyer plan: {plan.m} terms synthesised and planned in {time.perf_counter() - t0:.2f} s")
        else:
            plan = pcm.Plan(wins, p.h, batch=p.batch, product_convolution=args.workload in PRODUCT_CONVOLUTION,
                            full_grid=args.workload in FULL_GRID)
        u = torch.from_numpy(p.u).to(dev)
        jobs.append((p, plan, u, torch.empty_like(u), torch.empty_like(u)))
        c = algorithmic_counts(p, plan.info())
        counts["flops_per_step"] += c["flops_per_step"]
        counts["bytes_per_step"] += c["bytes_per_step"]
        for key in ("kernel_flops", "kernel_bytes"):
            for k, v in c[key].items():
                counts[key][k] = counts[key].get(k, 0.0) + v
    samples_per_step = sum(2 * p.batch * p.n_total for p in probs)

    def step_plans():
        for _, plan, u, y, x in jobs:
            plan.apply(u, out=y)
            plan.apply_adjoint(u, out=x)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    extra = {}
    step = step_plans
    batch = None
    if args.workload == "c4":
        # all instances in one graph launch per direction, against the loop of single plans
        batch = pcm.Batch([j[1] for j in jobs], persistent=args.persistent)
        b_in, b_y, b_x = [j[2] for j in jobs], [j[3] for j in jobs], [j[4] for j in jobs]

        def step_batch():
            batch.apply(b_in, outputs=b_y)
            batch.apply_adjoint(b_in, outputs=b_x)
        if not args.no_compare:
            extra["single_plans_ms_per_step"] = round(timed(step_plans, max(args.steps // 4, 2)), 5)
        step = step_batch
    elif args.workload == "c5ad":
        from paper_1604_04374_amd.autograd import ExpansionOperator
        p0 = probs[0]
        op = ExpansionOperator((p0.w_rows, p0.w_cols), p0.h, batch=1)
        u_ad = jobs[0][2].clone().requires_grad_(True)
        f_ad = torch.randn_like(u_ad)

        def step_autograd():
            u_ad.grad = None
            op.spec.grad = None
            loss = 0.5 * torch.sum((op(u_ad) - f_ad) ** 2)
            loss.backward()
        if not args.no_compare:
            extra["plain_ms_per_step"] = round(timed(step_plans, args.steps), 5)
        step = step_autograd

    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    # HIP events on torch's current stream, the stream the library launches on
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    event_ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = samples_per_step / (ms_per_step * 1e-3)

    cold_ms = None
    if args.cold_steps > 0:
        # every step starts with caches holding none of its data: a 1 GiB
        # write (4x the Infinity Cache) on the same stream just before it
        log(f"[bench] {args.cold_steps} cold steps")
        flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.cold_steps)]
        for i, (e0, e1) in enumerate(ev):
            flush.fill_(float(i))
            e0.record()
            step()
            e1.record()
        torch.cuda.synchronize()
        cold_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        del flush
    copy_gbps = measure_copy_gbps(torch, dev)

    roofline = None
    kernels = {}
    if not args.no_trace and step is step_plans:
        log(f"[bench] per-kernel event pass ({args.steps} steps)")
        for _, plan, _, _, _ in jobs:
            plan.set_tracing(True)
            plan.trace_reset()
        for _ in range(args.steps):
            step()
        for _, plan, _, _, _ in jobs:
            for k, v in plan.trace_stats().items():
                agg = kernels.setdefault(k, {"launches": 0, "total_ms": 0.0})
                agg["launches"] += v["launches"]
                agg["total_ms"] += v["total_ms"]
            plan.set_tracing(False)
        traced_total = sum(v["total_ms"] for v in kernels.values())
        for k, v in kernels.items():
            v["avg_ms"] = v["total_ms"] / max(v["launches"], 1)
            v["launches_per_step"] = v["launches"] / args.steps
            v["share"] = v["total_ms"] / traced_total if traced_total > 0 else None
            per_launch = v["launches"] / args.steps
            v["pass_bytes_per_launch"] = counts["kernel_bytes"].get(k, 0.0) / per_launch if per_launch else 0.0
            v["alg_flops_per_launch"] = counts["kernel_flops"].get(k, 0.0) / per_launch if per_launch else 0.0
            v["traffic_per_launch"] = read_traffic(k, args.workload, probs[0].ndim)
    hbm_gbps = counts["bytes_per_step"] / (ms_per_step * 1e-3) / 1e9
    if probs[0].ndim == 1 and kernels:
        # VALU-bound: the dominant kernel's algorithmic FP32 rate
        name, st = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
        t_s = st["avg_ms"] * 1e-3
        flops = st["alg_flops_per_launch"]
        achieved = flops / t_s / 1e12
        roofline = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                    "traffic": st["traffic_per_launch"],
                    "avg_launch_ms": round(st["avg_ms"], 5), "flops_per_launch": flops,
                    "bytes_per_launch": st["pass_bytes_per_launch"]}
        if roofline["traffic"] and roofline["bytes_per_launch"] > 0:
            roofline["traffic_ratio"] = round(roofline["traffic"] / roofline["bytes_per_launch"], 2)
    elif probs[0].ndim == 2:
        # HBM-bound: the whole step (every launch of both directions) moving
        # the method's algorithmic bytes, timed with HIP events on the launch
        # stream around the timed region
        achieved = counts["bytes_per_step"] / (event_ms_per_step * 1e-3) / 1e9
        roofline = {"bound": "hbm",
                    "kernel": "whole step (every launch of H_m u and H_m^* u)" if step is step_plans
                    else "whole step (graph or autograd launches)",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": read_traffic("step", args.workload, 2),
                    "bytes_per_step": counts["bytes_per_step"], "event_ms_per_step": round(event_ms_per_step, 5),
                    "frac_of_copy": round(achieved / copy_gbps, 4)}
        if roofline["traffic"]:
            roofline["traffic_ratio"] = round(roofline["traffic"] / counts["bytes_per_step"], 2)
    p = probs[0]
    B = p.batch
    _, _, _, y, x = jobs[0]

    cpu = None
    err = None
    if args.cpu_seconds > 0:
        from oracle import expansion as ex
        log("[bench] CPU oracle baseline")
        errs = []
        tc = 0.0
        n_sig = 0
        done_samples = 0
        passes = 0
        total_sig = sum(q.batch for q in probs)
        refs = {}
        # whole passes over the workload until the budget is spent (the first
        # pass also checks the GPU outputs); a budget shorter than one pass
        # stops inside it
        while tc < args.cpu_seconds:
            for qi, (q, _, _, yq, xq) in enumerate(jobs):
                if tc >= args.cpu_seconds and n_sig > 0:
                    break
                if qi not in refs:
                    if args.workload == "c2meyer":
                        from oracle import wavelets as wv
                        lam, mu, c = q.extra["meyer"]
                        _, w64, h64 = wv.meyer_expansion(lam, mu, c.astype(np.float64), q.shape[0],
                                                         wv.daubechies(2), MEYER_LEVELS)
                    else:
                        w64 = q.dense_windows()
                        h64 = q.h.astype(np.float64)
                    refs[qi] = (w64, h64, yq.cpu().numpy(), xq.cpu().numpy())
                w64, h64, y_gpu, x_gpu = refs[qi]
                for b in range(q.batch):
                    if tc >= args.cpu_seconds and n_sig > 0:
                        break
                    uu = q.u[b:b + 1].astype(np.float64)
                    c0 = time.perf_counter()
                    if args.workload in PRODUCT_CONVOLUTION:
                        ry = ex.apply_pc_fft(uu, w64, h64)
                        rx = ex.adjoint_pc_fft(uu, w64, h64)
                    else:
                        ry = ex.apply_fft(uu, w64, h64)
                        rx = ex.adjoint_fft(uu, w64, h64)
                    tc += time.perf_counter() - c0
                    if passes == 0:
                        errs.append(float(np.linalg.norm(y_gpu[b] - ry[0]) / np.linalg.norm(ry[0])))
                        errs.append(float(np.linalg.norm(x_gpu[b] - rx[0]) / np.linalg.norm(rx[0])))
                    n_sig += 1
                    done_samples += 2 * q.n_total
            passes += 1
        cpu = {"value": round(done_samples / tc, 1), "unit": "samples/s", "cores": ex.workers(),
               "kind": "oracle",
               "sample": f"{n_sig} signal evaluations over the workload's {total_sig} signals "
                         f"({n_sig / total_sig:.2f} passes), forward + adjoint, float64 FFT form (scipy.fft, "
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
        "config": {"workload": WORKLOADS[args.workload], "key": args.workload, "plans": len(probs),
                   "batch": B, "shape": list(p.shape), "m": p.m},
        "roofline": roofline,
        "hbm": {"alg_bytes_per_step": counts["bytes_per_step"], "achieved_GBps": round(hbm_gbps, 1),
                "peak_GBps": HBM_PEAK_GBPS, "frac": round(hbm_gbps / HBM_PEAK_GBPS, 4),
                "copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(hbm_gbps / copy_gbps, 4)},
        "cold_ms_per_step": None if cold_ms is None else round(cold_ms, 5),
        "alg_tflops": round(counts["flops_per_step"] / (ms_per_step * 1e-3) / 1e12, 3),
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "launches_per_step": v["launches_per_step"],
                        "share": None if v["share"] is None else round(v["share"], 3),
                        "pass_bytes_per_launch": v["pass_bytes_per_launch"],
                        "traffic_per_launch": v["traffic_per_launch"]} for k, v in kernels.items()},
        "tuning": "rules only (--no-tuning)" if args.no_tuning else "tuning table",
        "max_rel_l2_vs_oracle": err,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)
    if batch is not None:
        batch.destroy()
    for _, plan, _, _, _ in jobs:
        plan.destroy()


def bench_construct(args, torch, pcm, dev):
    """Time pc_construct_project on the C2 TVIR band (one call = every lag row)."""
    import workloads as wl
    n, m = 65536, 32
    log("[bench] generating the TVIR band on the device")
    tv, lags = wl.gen.tvir_band_torch(n, wl.gen.c2_sigma, dev)
    W = wl.bspline_windows_1d(n, m, 3).astype(np.float32)
    Wd = torch.from_numpy(W).to(dev)
    rows = int(lags.shape[0])
    steps = max(1, min(args.steps, 10))
    log(f"[bench] {rows} rows x {n} positions; warmup {args.warmup}, timing {steps} calls")
    for _ in range(max(args.warmup, 1)):
        h = pcm.construct_project(tv, lags, Wd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h = pcm.construct_project(tv, lags, Wd)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    flops = 2.0 * rows * m * n + 2.0 * m * m * n
    tvir_bytes = rows * n * 4.0
    achieved = flops / (ms * 1e-3) / 1e12
    roofline = {"bound": "hbm", "kernel": "construct_project (whole call: GEMM, reduction, factorisation, solves)",
                "achieved": round(tvir_bytes / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(tvir_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                "mfma_tflops": round(achieved, 3), "mfma_frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4)}
    err = cpu = None
    if args.cpu_seconds > 0:
        # the oracle's projection on consecutive chunks of rows, within the
        # CPU budget; its agreement with the device result on those rows
        from oracle import construct
        W64 = W.astype(np.float64)
        tc, done, num, den = 0.0, 0, 0.0, 0.0
        hc = h.cpu().numpy()
        for r0 in range(0, rows, 2048):
            if tc >= args.cpu_seconds:
                break
            sub = tv[r0:r0 + 2048].cpu().numpy().astype(np.float64)
            c0 = time.perf_counter()
            ref = construct.project(sub, W64)
            tc += time.perf_counter() - c0
            got = hc[:, lags[r0:r0 + 2048]]
            num += float(np.sum((got - ref) ** 2))
            den += float(np.sum(ref ** 2))
            done += sub.shape[0]
        err = float(np.sqrt(num / den))
        cpu = {"value": round(done / tc, 1), "unit": "rows/s", "cores": __import__("oracle").expansion.workers(),
               "kind": "oracle", "sample": f"{done} of {rows} rows, float64 NumPy projection, {tc:.2f} s"}
    line = {
        "metric": "TVIR lag rows projected per second (n=65536, m=32 cubic B-spline windows)",
        "value": round(rows / (ms * 1e-3), 1), "unit": "rows/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (FP32 MFMA products, float64 sums of chunks and solves)",
        "data": "synthetic", "config": {"workload": WORKLOADS["c2proj"], "key": "c2proj", "rows": rows,
                                        "n": n, "m": m},
        "roofline": roofline, "alg_tflops": round(achieved, 3), "max_rel_l2_vs_oracle": err, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
