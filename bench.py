"""Benchmark of the chi^2 hot path on one MI355X.

Workload (one step): the 16-detector histogram set of 16 x 65,536 bins
(0.0002 us bins; shared A, lambda, nu and a static Gaussian Kubo-Toyabe
component, per-detector N0, Nbkg and phase: 52 parameters) with

  * one cost + analytic-gradient evaluation at a parameter vector, and
  * the 2P = 104-vector central-difference stencil that checks that gradient,
    evaluated in one batched launch.

That is 105 x 1,048,576 bin evaluations per step.  Inputs are resident in HBM
before the timed region; the value is whole-step bin throughput (Gbin/s).

Also reported: the dominant kernel's roofline position (HIP-event timing of
each launch on the stream it runs on), single-evaluation latency, and the FP64
CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-calib]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 vector
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
# Algorithmic FP64 flops per bin of the cost pass on this theory (FMA = 2):
# lifetime step 1, damped rotation 6, Kubo-Toyabe step and polynomial 9,
# asymmetry 3, histogram model 3, chi^2 term 4, accumulation 1.
FLOPS_PER_BIN_CHI2 = 27
BYTES_PER_BIN = 4         # one FP32 count streamed per bin evaluation


def _workload(api, ctx):
    """The 16 x 65536 set: counts drawn from the library's own model values."""
    import synth

    cfg = synth.config_c2()
    th_d, p_true = cfg["theory"], cfg["p_true"]
    th = api.Theory(ctx, th_d)
    zero = [np.zeros(h["n_bins"]) for h in cfg["histos"]]
    grid = api.Data(ctx, cfg["histos"], zero)
    means = api.model_eval(ctx, grid, th, p_true)
    n = cfg["histos"][0]["n_bins"]
    counts = synth.draw_counts(means, cfg["rng"]).reshape(len(cfg["histos"]), n)
    data = api.Data(ctx, cfg["histos"], list(counts))
    return cfg, th, data, counts


def _stencil(p, rel=1e-4):
    P = []
    for k in range(p.size):
        h = rel * max(abs(p[k]), 1.0)
        for sgn in (1.0, -1.0):
            q = p.copy()
            q[k] += sgn * h
            P.append(q)
    return np.array(P)


def _cpu_baseline(cfg, counts, stencil, budget_s=12.0):
    """The FP64 oracle as it is, timed on a bounded sample of the stencil."""
    from oracle import model

    t0 = time.perf_counter()
    done = 0
    bins = 0
    for q in stencil:
        model.cost(cfg["theory"], cfg["histos"], list(counts), q)
        done += 1
        bins += sum(h["n_bins"] for h in cfg["histos"])
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": bins / dt / 1e9, "unit": "Gbin/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the {len(stencil)} stencil vectors over all 16 x 65536 bins "
                      f"({bins} bin evaluations, {dt:.1f} s, numpy + math.fsum, one thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 256 MiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.copy_calib:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": x.numel() * 4}))
        return

    from paper_1604_02334_amd import api

    ctx = api.Context(0)
    cfg, th, data, counts = _workload(api, ctx)
    p0 = cfg["p_true"] * (1.0 + 1e-3 * np.cos(np.arange(cfg["p_true"].size)))
    stencil = _stencil(p0)
    n_bins = data.n_bins
    dev = torch.device("cuda:0")
    p_dev = torch.tensor(p0[None], dtype=torch.float64, device=dev)
    s_dev = torch.tensor(stencil, dtype=torch.float64, device=dev)
    st = ctx.torch_stream

    def step(ev=None):
        api.chi2_grad(ctx, data, th, p_dev)
        if ev is not None:
            ev[0].record(st)
        c = api.chi2_eval(ctx, data, th, s_dev)
        if ev is not None:
            ev[1].record(st)
        return c

    # measured tile / anchor choice for both launches (untimed)
    tune_eval = api.autotune(ctx, data, th, s_dev)
    tune_grad = api.autotune(ctx, data, th, p_dev, grad=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in evs])

    # single-vector latency (cost only, host in and out)
    host_p = p0[None]
    for _ in range(5):
        api.chi2_eval(ctx, data, th, host_p)
    t1 = time.perf_counter()
    for _ in range(50):
        api.chi2_eval(ctx, data, th, host_p)
    lat_us = (time.perf_counter() - t1) / 50 * 1e6

    bins_per_step = (1 + stencil.shape[0]) * n_bins
    ms_per_step = wall / args.steps * 1e3
    value = bins_per_step / (wall / args.steps) / 1e9
    k_ms = float(np.mean(kern_ms))
    k_bins = stencil.shape[0] * n_bins
    achieved = FLOPS_PER_BIN_CHI2 * k_bins / (k_ms * 1e-3) / 1e12
    out = {
        "metric": "chi2 Gbin/s (FP64 acc, 1e-10 rel)",
        "value": round(value, 3),
        "unit": "Gbin/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2_16x65536_grad_plus_104_vector_central_difference_stencil",
                   "histograms": 16, "bins_per_histogram": 65536, "params": 52,
                   "vectors_per_step": 1 + stencil.shape[0], "bins_per_step": bins_per_step},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "eval_kernel<chi2, cost, float>", "kernel_ms": round(k_ms, 5),
                     "flops_per_bin": FLOPS_PER_BIN_CHI2, "bins_per_launch": k_bins},
        "extra": {"stencil_kernel_gbin_s": round(k_bins / (k_ms * 1e-3) / 1e9, 2),
                  "tuned_stencil": {"tile": tune_eval[0], "anchor": tune_eval[1]},
                  "tuned_grad": {"tile": tune_grad[0], "anchor": tune_grad[1]},
                  "single_eval_host_latency_us": round(lat_us, 2)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(cfg, counts, stencil)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
