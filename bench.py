"""Benchmark of the KNN filtering hot path on one MI355X.

Workload (one step = one pass of the whole hot path over one frame): the
brain-like frame W 480 x H 380 (182,400 pixels), one-band image + 4-class
probability maps, K = 40, window +-14 rows at full width, lambda = 0.01, all
inputs resident in device memory before timing starts.  Each step runs the
whole filter (distances, top-K selection, averaging, argmax) in one kernel
launch and writes the filtered maps and the class map.

Prints one JSON line with the headline throughput (filtered pixels/s), per-frame
latency percentiles, the roofline of the filter kernel (measured with HIP
events on the launch stream) and the CPU oracle's throughput on a bounded
sample of the same frame.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--plan exhaustive|pruned]
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

METRIC = "filtered pixels/sec at K=40 (served vs plain); p50/p99 frame latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak (256 CU, 2.4 GHz)
FLOP_PER_PAIR = 8                 # 3 subtractions, 3 squares, 2 additions of Eq. 1


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plan", default="pruned", choices=["exhaustive", "pruned"])
    ap.add_argument("--tile-rows", type=int, default=2)
    ap.add_argument("--tile-cols", type=int, default=4)
    ap.add_argument("--waves", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    return ap.parse_args()


def cpu_baseline(spec, pc1, prob, target_s):
    """Oracle throughput on a bounded random sample of the frame's pixels."""
    import oracle

    nt = oracle.max_threads()
    H, W = spec.H, spec.W
    rng = np.random.default_rng(77)
    probe = rng.integers(0, H * W, 512)
    t0 = time.perf_counter()
    oracle.knn_pixels(pc1, prob, spec.K, spec.R, spec.lam, probe, with_nbr=False, nthreads=nt)
    dt = max(time.perf_counter() - t0, 1e-3)
    n = int(min(H * W, max(2048, 512 * target_s / dt)))
    pix = rng.integers(0, H * W, n)
    t0 = time.perf_counter()
    oracle.knn_pixels(pc1, prob, spec.K, spec.R, spec.lam, pix, with_nbr=False, nthreads=nt)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "pixels/s", "cores": nt, "kind": "oracle",
            "sample": f"{n} random pixels of the W480xH380 brain-like frame (K=40, +-14 rows), "
                      f"{dt:.1f} s on {nt} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); frames are "
              "independent, so several GPUs would each run this same single-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2404_10631_amd import _lib, inputs
    from paper_2404_10631_amd.frames import DeviceFrame, current_stream

    torch.cuda.set_device(0)
    spec = inputs.config1().frames[0]
    pc1, prob = spec.make()
    frame = DeviceFrame(pc1, prob, spec.K, spec.R, spec.lam, with_nbr=False)
    cf = frame.as_c()
    ctx = _lib.knnf_create(0)
    plan = {"search": 0 if args.plan == "exhaustive" else 1, "tile_rows": args.tile_rows,
            "tile_cols": args.tile_cols, "waves": args.waves}
    stream = current_stream()

    for _ in range(args.warmup):
        _lib.knnf_filter(ctx, cf, plan, stream)
    torch.cuda.synchronize()

    # latency: one frame at a time, events around each launch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for k in range(args.steps):
        starts[k].record()
        _lib.knnf_filter(ctx, cf, plan, stream)
        ends[k].record()
        ends[k].synchronize()
    lat_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])

    # throughput: K launches back to back
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        _lib.knnf_filter(ctx, cf, plan, stream)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kernel_ms = gpu_ms / args.steps
    px = spec.pixels
    value = px * args.steps / wall

    pairs = spec.pairs()
    achieved = pairs * FLOP_PER_PAIR / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": None,
                "kernel": "filter_frame_kernel", "kernel_ms": round(kernel_ms, 5),
                "work": f"{pairs} window pairs x {FLOP_PER_PAIR} FLOP"}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "pixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec_name(spec), "frames_per_step": 1, "H": spec.H, "W": spec.W,
                   "K": spec.K, "R": spec.R, "lambda": spec.lam, "classes": spec.C,
                   "plan": plan},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 5),
                       "p99": round(float(np.percentile(lat_ms, 99)), 5)},
        "roofline": roofline,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, pc1, prob, args.cpu_seconds)
    _lib.knnf_destroy(ctx)
    print(json.dumps(out), flush=True)


def spec_name(spec):
    return f"plain KNN filter, brain-like W{spec.W}xH{spec.H}, K={spec.K}, +-{spec.R} rows"


if __name__ == "__main__":
    main()
