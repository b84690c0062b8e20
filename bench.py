#!/usr/bin/env python3
"""Benchmark of the wavelet-transparency resolve on one MI355X.

One step is the whole path for one frame of the smoke workload (1920x1080, Poisson(64 g(x,y)) fragments per
pixel, g a seeded clipped blob field of mean 1, depth Normal(0.5, 0.1), alpha U[0.02, 0.1], unsorted stream,
rank 3, FP32 coefficients): screen-tile binning (wt_bin), then build + evaluate + resolve (wt_render_binned),
writing the frame's coefficients and its composite. Inputs are resident in HBM before the timed region.

Prints one JSON line: whole-job fragments/s, p50/p99 frame latency, the roofline of the dominant kernel
(timed with events on the library's stream) and the FP64 CPU oracle timed on a bounded sample of the same
frame on the host cores.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "resolved fragments/s (build+eval) 1080p×64 frag/px; % HBM peak; p99 ms"


def algorithmic_bytes(F, P, M, coeff_bytes):
    """Bytes the two-pass method must move for an unsorted stream (one visibility channel): the build reads
    pixel, depth, alpha (12 B/fragment); the evaluate reads pixel, depth, alpha, rgb (24 B/fragment); the
    coefficients are written and read once (2 s M B/pixel), the accumulation written and read (32 B/pixel) and
    the composite written (12 B/pixel)."""
    return F * (12 + 24) + P * (2 * coeff_bytes * M + 16 + 16 + 12)


def render_kernel_bytes(F, P, M, coeff_bytes):
    """Algorithmic bytes of the fused per-tile kernel: the build and evaluate reads of each binned fragment
    (tile-local pixel, depth, alpha: 12 B; plus rgb: 24 B), the coefficient store (s M B/pixel) and the
    composite store (12 B/pixel); the accumulation never leaves LDS."""
    return F * (12 + 24) + P * (coeff_bytes * M + 12)


def scatter_kernel_bytes(F):
    """Algorithmic bytes of the binning scatter: read the fragment (24 B) and write its binned copy (24 B)."""
    return F * 48


def cpu_baseline(f, fraction, seed):
    import oracle
    rng = np.random.default_rng(seed + 17)
    mask = rng.random(f.pixels) < fraction
    n = int(np.bincount(f.pixel, minlength=f.pixels)[mask].sum())
    t0 = time.perf_counter()
    oracle.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, mask=mask, want=("out",))
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "fragments/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle resolve of %d fragments: the pixels of a seeded %.0f%% sample of the same frame "
                      "(%.1f s wall)" % (n, 100 * fraction, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rank", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=("f32", "f16", "bf16"))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-fraction", type=float, default=0.1,
                    help="share of the frame's pixels the CPU oracle baseline resolves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus %d, WORLD_SIZE %d)"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2201_00094_amd as wt
    import synth

    t_gen = time.perf_counter()
    f = synth.frame_c2(seed=args.seed, rank=args.rank)
    gen_s = time.perf_counter() - t_gen
    print("bench: generated %s, %d fragments in %.1f s" % (f.name, f.count, gen_s), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = wt.FrameSpec(f.width, f.height, args.rank, 1, args.dtype)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb, device=dev)
    ws = wt.Workspace(spec, f.count, device=dev)
    coeffs = spec.new_coeffs(device=dev)
    out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        wt.bin(spec, fr, ws, stream=stream)
        wt.render_binned(spec, ws, f.bg, out, coeffs, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if wt.dropped_count(ws) != 0:
        raise RuntimeError("fragments were dropped from a clean stream")

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        wt.bin(spec, fr, ws, stream=stream)
        ev[k][1].record(stream)
        wt.render_binned(spec, ws, f.bg, out, coeffs, stream=stream)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    frame_ms = np.array([ev[k][0].elapsed_time(ev[k][2]) for k in range(K)])
    bin_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    render_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    ms_per_step = wall * 1e3 / K
    F, P, M = f.count, f.pixels, spec.M
    sbytes = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    b_alg = algorithmic_bytes(F, P, M, sbytes)
    b_render = render_kernel_bytes(F, P, M, sbytes)
    render_gbs = b_render / (render_ms.mean() * 1e-3) / 1e9

    line = {
        "metric": METRIC,
        "value": F * K / wall,
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "smoke 1920x1080, Poisson(64 g) fragments/px (unsorted stream), rank %d, %s "
                               "coefficient storage" % (args.rank, args.dtype),
                   "width": f.width, "height": f.height, "rank": args.rank, "coeff_dtype": args.dtype,
                   "fragments": F, "seed": args.seed},
        "p50_ms": float(np.percentile(frame_ms, 50)),
        "p99_ms": float(np.percentile(frame_ms, 99)),
        "phase_ms": {"bin": float(bin_ms.mean()), "render": float(render_ms.mean())},
        "path_alg_bytes": b_alg,
        "path_hbm_frac": b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": "k_render", "achieved": render_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": render_gbs / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": b_render},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(f, args.cpu_fraction, args.seed)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
