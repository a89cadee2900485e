"""Benchmark: events/s reconstructed on one MI355X.

Workload (the detector the headline metric is quoted on): 37 photomultipliers
on a hexagonal grid (pitch 30 mm), r-z LRF as a 24 x 16 cubic B-spline,
10 M flood-field events uniform in r < 90 mm and z in [0, 50] mm with
E_tot uniform in [500, 2000] photoelectrons, Poisson counts; contracting grid
7 x 7 x 7 nodes, 8 iterations, shrink 0.5, start at the centroid.  Events are
drawn on the GPU by the library's own generator (synthetic data) and are
resident in HBM before the timed region.

One step = one reconstruction of the whole 10 M-event batch.  Prints one JSON
line.  The CPU baseline times the FP64 oracle on a bounded sample of the same
events on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (packed), published
# canonical FP32 operations per (node, sensor) evaluation, ML statistic:
# distance 5 + sqrt 1 + interval 2 + cubic 6 + clamp 1 + S 2 + log 1 + n*log 2
FLOP_PER_EVAL_ML = 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=24_000,
                    help="events for the oracle CPU baseline (0 = skip)")
    ap.add_argument("--seed", type=int, default=160207247)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    return ap.parse_args()


def copy_probe():
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_copy": a.numel() * 4,
                      "copy_probe_bytes_written_per_copy": a.numel() * 4}))


def cpu_baseline(wl, sig_host):
    import oracle
    threads = os.cpu_count() or 1
    oracle.build()
    t0 = time.perf_counter()
    oracle.reconstruct(wl.lrf, wl.grid, sig_host, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": len(sig_host) / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {len(sig_host)} events of the benchmark batch, FP64 C oracle, "
                      f"{threads} threads, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import torch
    import workloads as W
    from paper_1602_07247_amd import ants

    wl = W.workload(2)
    n = args.events
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lrf = ants.LrfSet(wl.lrf)
    cfg = ants.grid_cfg(wl.grid)
    sig, truth = ants.generate(lrf, ants.gen_cfg(wl.events), n, args.seed)
    out = ants.alloc_out(n)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ants.reconstruct(lrf, cfg, sig, out=out, stream=stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        ants.reconstruct(lrf, cfg, sig, out=out, stream=stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))

    ms_per_step = 1e3 * wall / args.steps
    evs = n / (wall / args.steps)
    evals = wl.grid.nodes[0] * wl.grid.nodes[1] * wl.grid.nodes[2] * 37 * wl.grid.iterations
    flops = n * evals * FLOP_PER_EVAL_ML
    achieved = flops / (kern_ms * 1e-3) / 1e12

    t = truth.cpu().numpy()
    dx = out["x"].cpu().numpy() - t[:, 0]
    dy = out["y"].cpu().numpy() - t[:, 1]
    sigma_xy = float(np.sqrt(0.5 * np.mean(dx * dx + dy * dy)))
    status = out["status"].cpu().numpy()

    rec = {
        "metric": "events/s reconstructed (plain grid vs NN-seeded) at equal sigma_xy, 1 MI355X",
        "value": evs, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic (flood-field events drawn on the GPU from the LRF model)",
        "config": {"workload": "hex37 r-z LRF, 10M events, plain contracting grid 7x7x7 x 8 "
                               "iterations, ML statistic, centroid start",
                   "events": n, "sensors": 37, "grid": list(wl.grid.nodes),
                   "iterations": wl.grid.iterations},
        "sigma_xy_mm": sigma_xy,
        "bad_status_events": int(((status & 7) != 0).sum()),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "cg_kernel<RZ,ML,NT=6>", "kernel_ms": kern_ms,
                     "flop_per_launch": flops},
    }
    if args.cpu_sample > 0:
        m = min(args.cpu_sample, n)
        rec["cpu_baseline"] = cpu_baseline(wl, sig[:m].cpu().numpy())
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
