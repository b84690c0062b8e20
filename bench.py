#!/usr/bin/env python3
"""Benchmark of the wavelet-transparency resolve on one MI355X.

One step is the whole path for one frame of the smoke workload (1920x1080, Poisson(64 g(x,y)) fragments per
pixel, g a seeded clipped blob field of mean 1, depth Normal(0.5, 0.1), alpha U[0.02, 0.1], unsorted stream,
rank 3, FP32 coefficients): screen-tile binning (wt_bin_count, wt_bin_scatter), then build + evaluate + resolve
(wt_render_binned), writing the frame's coefficients and its composite. Inputs are resident in HBM before the
timed region.

Prints one JSON line: whole-job fragments/s, p50/p99 frame latency, the roofline of the dominant kernel
(timed with events on the library's stream) and the FP64 CPU oracle timed on a bounded sample of the same
frame on the host cores.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
LDS_F64_ATOMIC_CEILING = 3.0  # ds_add_f64 per compute unit per clock, random addresses (measured probe)
METRIC = "resolved fragments/s (build+eval) 1080p×64 frag/px; % HBM peak; p99 ms"
CSRC = os.path.join(ROOT, "paper_2201_00094_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_smoke1080p.json")
# short kernel names used in the JSON line -> prefix of the demangled name in rocprofv3's output
KERNEL_PREFIX = {"k_scatter_staged": "void wt::k_scatter_staged<", "k_render": "void wt::k_render<",
                 "k_hist_lds": "void wt::k_hist_lds<", "k_render_temporal": "void wt::k_render_temporal<"}


def sources_digest():
    """SHA-256 over the kernel sources: HBM counter readings are valid only for the sources they were taken on."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if p.endswith((".hip", ".h")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def workload_key(args):
    """Key of a smoke-frame configuration in the traffic summary."""
    return "r%d_%s" % (args.rank, args.dtype) + ("_tight" if args.tight else "") + \
        ("_temporal" if args.temporal else "")


def measured_traffic(kernel, key):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, or None when the summary was taken
    on other kernel sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_digest():
        return None
    return t.get("workloads", {}).get(key, {}).get(kernel)


def algorithmic_bytes(F, P, C, coeff_px):
    """Bytes the two-pass method must move for an unsorted stream with C visibility channels: the build reads
    pixel, depth, alpha (8 + 4C B/fragment); the evaluate reads them and rgb (20 + 4C B/fragment); the
    coefficients are written and read once (2 x coeff_px B/pixel: s C M, or 4 M for E5B9G9R9), the accumulation
    written and read (16 B/pixel at C = 1, 32 at C = 3, each way) and the composite written (12 B/pixel).
    One channel: F 36 + P (2 s M + 44)."""
    acc = 16 if C == 1 else 32
    return F * ((8 + 4 * C) + (20 + 4 * C)) + P * (2 * coeff_px + 2 * acc + 12)


def render_kernel_bytes(F, P, C, coeff_px):
    """Algorithmic bytes of the fused per-tile kernel: the build and evaluate reads of each binned fragment
    (tile-local pixel, depth, alpha: 8 + 4C B; plus rgb: 20 + 4C B), the coefficient store and the composite
    store (12 B/pixel); the accumulation never leaves LDS."""
    return F * ((8 + 4 * C) + (20 + 4 * C)) + P * (coeff_px + 12)


def temporal_bytes(F, P, C, coeff_px):
    """Algorithmic bytes of the one-pass render against the previous frame (path and kernel alike): each
    fragment read once (tile-local pixel, depth, alpha, rgb: 20 + 4C B), the previous coefficients read and this
    frame's written (2 x coeff_px B/pixel), the composite written (12 B/pixel)."""
    return F * (20 + 4 * C) + P * (2 * coeff_px + 12)


def scatter_kernel_bytes(F, C):
    """Algorithmic bytes of the binning scatter: read the fragment (20 + 4C B) and write its binned record
    (tile-local pixel, depth, alpha, rgb: 20 + 4C B); 48 B at C = 1."""
    return F * 2 * (20 + 4 * C)


def roofline(path_bytes, kernel, kernel_ms, traffic):
    """Roofline object of the benchmark line. achieved = the path's algorithmic bytes per frame (the per-fragment and
    per-pixel figures of ``algorithmic_bytes``, times the frame's fragments and pixels, which one launch of the
    dominant kernel processes) over that kernel's mean launch time; frac = achieved / the published 8 TB/s. The
    binned copy that the scatter writes and the tile kernel reads back is not algorithmic and earns nothing here.
    traffic = the kernel's HBM bytes per launch from the committed counter summary (None when it was taken on other
    sources)."""
    achieved = path_bytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": path_bytes,
            "avg_ms": kernel_ms}


def cpu_model():
    """The host CPU's model name (what lscpu reports as "Model name"), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(fn, min_seconds, max_reps):
    reps, dt = 0, 0.0
    while reps < max_reps and (reps == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        fn()
        dt += time.perf_counter() - t0
        reps += 1
    return reps, dt


def cpu_baseline(f, fraction, seed, single_fraction=0.05, min_seconds=4.0, max_reps=4):
    """The FP64 oracle on the host cores, three legs on seeded pixel samples of the same frame (each repeated until
    about ``min_seconds`` of wall time): the wavelet resolve on every core (OpenMP over pixels; the headline
    ``value``), the same on one thread, and the exact sorted A-buffer on every core. Thread counts are passed
    explicitly: the oracle's thread setting persists between calls."""
    import oracle
    rng = np.random.default_rng(seed + 17)
    u = rng.random(f.pixels)
    per_px = np.bincount(f.pixel, minlength=f.pixels)
    n_all = oracle.num_threads()
    legs = {}

    def leg(name, frac, threads, fn):
        mask = u < frac
        n = int(per_px[mask].sum())
        reps, dt = _time_oracle(lambda: fn(mask, threads), min_seconds, max_reps)
        legs[name] = {"value": n * reps / dt, "unit": "fragments/s", "threads": threads,
                      "sample": "%.0f%% of the pixels (%d fragments), %d time(s), %.1f s wall" % (100 * frac, n, reps,
                                                                                                   dt)}

    def wavelet(mask, threads):
        oracle.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=f.channels,
                       mask=mask, want=("out",), threads=threads)

    def abuf(mask, threads):
        oracle.abuffer(f.width, f.height, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=f.channels, mask=mask,
                       threads=threads)

    leg("wavelet_all_cores", fraction, n_all, wavelet)
    leg("wavelet_one_thread", min(fraction, single_fraction), 1, wavelet)
    leg("abuffer_all_cores", fraction, n_all, abuf)
    head = legs["wavelet_all_cores"]
    return {"value": head["value"], "unit": "fragments/s", "cores": n_all, "kind": "oracle",
            "sample": "FP64 oracle wavelet resolve (build, cells, interpolation, composite) of the same frame on %d "
                      "threads: %s; legs below: one thread, and the exact A-buffer timed separately" % (n_all,
                                                                                                      head["sample"]),
            "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "legs": legs}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rank", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=("f32", "f16", "bf16", "e5b9g9r9"))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-fraction", type=float, default=1.0,
                    help="share of the frame's pixels the CPU oracle baseline resolves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="frame",
                    choices=("frame", "serve", "copy", "traffic", "precision", "chromatic", "overlap"),
                    help="frame: the headline single-frame step (default); serve: the continuous-batching trace; "
                         "copy: a plain device copy of known size (calibrates the HBM byte counters); traffic: "
                         "turn rocprofv3 FETCH_SIZE / WRITE_SIZE collections into the committed traffic summary; "
                         "precision: the glass + particles frame (3840x2160, three channels) with every coefficient "
                         "storage, timed, with errors against the FP64 oracle and the exact A-buffer")
    ap.add_argument("--tight", action="store_true", help="per-pixel depth bounds (WT_TIGHT_DEPTH)")
    ap.add_argument("--temporal", action="store_true",
                    help="one pass per frame against the previous frame's coefficients (WT_TEMPORAL)")
    ap.add_argument("--workload", default="smoke", choices=("smoke", "glass"),
                    help="frame mode: smoke (1920x1080, one visibility channel; the headline) or glass "
                         "(3840x2160 glass + particles, three visibility channels)")
    ap.add_argument("--offsets", default="smooth", choices=("smooth", "noise"),
                    help="chromatic mode: refraction offsets as a smooth field or independent per-pixel noise")
    ap.add_argument("--sample-pixels", type=int, default=4000, help="precision mode: pixels checked by the oracle")
    ap.add_argument("--pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="traffic mode: rocprofv3 output folders of the frame and copy runs")
    ap.add_argument("--pmc-command", default="", help="traffic mode: the command the counters were taken with")
    ap.add_argument("--requests", type=int, default=500, help="serve mode: requests per trace")
    ap.add_argument("--trace", help="overlap mode: kernel_trace.csv of a rocprofv3 --kernel-trace run of --mode serve")
    ap.add_argument("--load", default="0.5,0.8,0.95",
                    help="serve mode: arrival rates as shares of the solo capacity (comma-separated sweep)")
    ap.add_argument("--budget-gb", type=float, default=96.0,
                    help="serve mode: HBM admission budget (default: room for five 3840x2160 requests)")
    ap.add_argument("--slots", type=int, default=3, help="serve mode: concurrent requests (HIP streams)")
    ap.add_argument("--policy", choices=("fifo", "sjf"), default="sjf",
                    help="serve mode: admission order (fewest fragments first with a bounded bypass, the default; or "
                         "first come first)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus %d, WORLD_SIZE %d)"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    if args.mode == "serve":
        return run_serve(args)
    if args.mode == "copy":
        return run_copy(args)
    if args.mode == "overlap":
        return run_overlap(args)
    if args.mode == "traffic":
        return run_traffic(args)
    if args.mode == "precision":
        return run_precision(args)
    if args.mode == "chromatic":
        return run_chromatic(args)

    import torch

    import paper_2201_00094_amd as wt
    import synth

    t_gen = time.perf_counter()
    glass = args.workload == "glass"
    f = synth.frame_c3(seed=args.seed, rank=args.rank) if glass else synth.frame_c2(seed=args.seed, rank=args.rank)
    gen_s = time.perf_counter() - t_gen
    print("bench: generated %s, %d fragments in %.1f s" % (f.name, f.count, gen_s), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = wt.FrameSpec(f.width, f.height, args.rank, f.channels, args.dtype, args.tight, args.temporal)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb, device=dev)
    ws = wt.Workspace(spec, f.count, device=dev)
    # one-pass mode: this frame's coefficients go to one buffer while the previous frame's are read from the
    # other; the two swap every frame
    bufs = [spec.new_coeffs(device=dev), spec.new_coeffs(device=dev) if args.temporal else None]
    out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def render():
        if args.temporal:
            wt.render_temporal_binned(spec, ws, f.bg, out, prev=bufs[1], coeffs=bufs[0], stream=stream)
            bufs.reverse()
        else:
            wt.render_binned(spec, ws, f.bg, out, bufs[0], stream=stream)

    def step():
        wt.bin_count(spec, fr, ws, stream=stream)
        wt.bin_scatter(spec, fr, ws, stream=stream)
        render()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if wt.dropped_count(ws) != 0:
        raise RuntimeError("fragments were dropped from a clean stream")

    K = args.steps
    # events on the library's stream between its calls: count (hist + scan), scatter, render (one kernel each
    # for the last two)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        wt.bin_count(spec, fr, ws, stream=stream)
        ev[k][1].record(stream)
        wt.bin_scatter(spec, fr, ws, stream=stream)
        ev[k][2].record(stream)
        render()
        ev[k][3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    frame_ms = np.array([ev[k][0].elapsed_time(ev[k][3]) for k in range(K)])
    count_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    scatter_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    render_ms = np.array([ev[k][2].elapsed_time(ev[k][3]) for k in range(K)])
    ms_per_step = wall * 1e3 / K
    F, P, M, C = f.count, f.pixels, spec.M, f.channels
    coeff_px = 4 * M if args.dtype == "e5b9g9r9" else {"f32": 4, "f16": 2, "bf16": 2}[args.dtype] * C * M
    if args.temporal:
        b_alg = temporal_bytes(F, P, C, coeff_px)
        models = {"k_render_temporal": (temporal_bytes(F, P, C, coeff_px), float(render_ms.mean()))}
    else:
        b_alg = algorithmic_bytes(F, P, C, coeff_px)
        models = {"k_render": (render_kernel_bytes(F, P, C, coeff_px), float(render_ms.mean()))}
    models["k_scatter_staged"] = (scatter_kernel_bytes(F, C), float(scatter_ms.mean()))
    dom = max(models, key=lambda k: models[k][1])
    dom_ms = models[dom][1]
    roof = roofline(b_alg, dom, dom_ms, None if glass else measured_traffic(dom, workload_key(args)))
    # each kernel's own byte model (what it reads and writes) over its own time: how close each runs to the memory
    # system's rate, which is not the method's roofline (the binning's bytes are not algorithmic)
    kernel_rates = {k: {"model_bytes": by, "ms": ms, "GBps": by / (ms * 1e-3) / 1e9,
                        "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS} for k, (by, ms) in models.items()}

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
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": ("glass + particles 3840x2160, 2-4 glass layers + Poisson(24) particles/px, three "
                                "visibility channels" if glass else
                                "smoke 1920x1080, Poisson(64 g) fragments/px") +
                               " (unsorted stream), rank %d, %s coefficient storage%s%s" % (
                                   args.rank, args.dtype, ", per-pixel depth bounds" if args.tight else "",
                                   ", one pass against the previous frame's coefficients" if args.temporal else ""),
                   "width": f.width, "height": f.height, "rank": args.rank, "coeff_dtype": args.dtype,
                   "fragments": F, "seed": args.seed},
        "p50_ms": float(np.percentile(frame_ms, 50)),
        "p99_ms": float(np.percentile(frame_ms, 99)),
        "phase_ms": {"count": float(count_ms.mean()), "scatter": float(scatter_ms.mean()),
                     "render": float(render_ms.mean())},
        "path_alg_bytes": b_alg,
        "path_hbm_frac": b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": roof,
        "kernel_rates": kernel_rates,
        "binning_rate_frac": kernel_rates["k_scatter_staged"]["frac"],
    }
    # coefficient and colour updates of the tile kernel: LDS FP64 atomics, 2 per channel for the endpoint masses
    # and 3 for the colour sums per fragment (the clock and CU count are the published ones; the ceiling is what a
    # random-address ds_add_f64 probe sustained on this GPU)
    n_at = F * (2 * C + 3)
    at_s = n_at / (float(render_ms.mean()) * 1e-3)
    per_cu_clk = at_s / (256 * 2.4e9)
    line["atomics"] = {"kind": "LDS ds_add_f64 in the tile kernel (%d per fragment)" % (2 * C + 3),
                       "per_launch": n_at, "per_s": at_s, "per_cu_per_clock": per_cu_clk,
                       "ceiling_per_cu_per_clock": LDS_F64_ATOMIC_CEILING,
                       "frac": per_cu_clk / LDS_F64_ATOMIC_CEILING}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(f, args.cpu_fraction, args.seed)
    print(json.dumps(line))


def run_chromatic(args):
    """The chromatic-aberration composite alone (wt_resolve_chromatic) on a whole frame: 1920x1080 with one
    visibility channel, or 3840x2160 with three (--workload glass); seeded accumulation, background image and
    refraction offsets resident in HBM; five taps, dispersion 0.5. The offsets are a smooth field of up to 20 px
    (refraction through curved glass varies smoothly across the screen) plus U[-1, 1] px of per-pixel noise, or
    U[-20, 20] px independently per pixel with --offsets noise (no locality between neighbours). Algorithmic bytes
    per pixel: the accumulation (16 or 32 B), the offset (8 B), the background texel once (12 B) and the composite
    (12 B)."""
    import torch

    import paper_2201_00094_amd as wt
    glass = args.workload == "glass"
    W, H, C = (3840, 2160, 3) if glass else (1920, 1080, 1)
    P = W * H
    rng = np.random.default_rng(args.seed)
    spec = wt.FrameSpec(W, H, args.rank, C)
    dev = torch.device("cuda:0")
    acc = torch.from_numpy(rng.random((P, spec.accum_width), dtype=np.float32)).to(dev)
    bg = torch.from_numpy(rng.random((P, 3), dtype=np.float32)).to(dev)
    if args.offsets == "noise":
        off_np = rng.uniform(-20, 20, (P, 2))
    else:
        y, x = np.divmod(np.arange(P), W)
        off_np = np.stack([20 * np.sin(2 * np.pi * (3 * x / W + 0.5 * y / H)),
                           20 * np.cos(2 * np.pi * (2 * y / H + 0.3 * x / W))], axis=1) + rng.uniform(-1, 1, (P, 2))
    off = torch.from_numpy(off_np.astype(np.float32)).to(dev)
    out = torch.empty((P, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        wt.resolve_chromatic(spec, acc, bg, off, 0.5, 5, out, stream=stream)
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(K):
        wt.resolve_chromatic(spec, acc, bg, off, 0.5, 5, out, stream=stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    by = P * (4 * spec.accum_width + 8 + 12 + 12)
    gbs = by / (ms.mean() * 1e-3) / 1e9
    print(json.dumps({"mode": "chromatic", "width": W, "height": H, "channels": C, "taps": 5, "dispersion": 0.5,
                      "offsets": args.offsets,
                      "ms": float(ms.mean()), "p99_ms": float(np.percentile(ms, 99)), "pixels_per_s": P / (ms.mean() * 1e-3),
                      "roofline": {"bound": "hbm", "kernel": "k_resolve_chromatic", "achieved": gbs,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                   "alg_bytes_per_launch": by}}))


def run_precision(args):
    """One frame per coefficient storage, timed, with the composite's error against the FP64 oracle at exact storage,
    against the exact A-buffer, and against the plain FP32 storage form, over the whole frame or a seeded pixel
    sample (``--sample-pixels``; 0 = every pixel). ``--workload smoke``: the headline frame (1920x1080, one
    channel), storage f32/f16/bf16. ``--workload glass``: glass + particles, 3840x2160, 2-4 glass layers with
    per-channel alpha plus Poisson(24) particles, three visibility channels, storage f32/f16/bf16/e5b9g9r9."""
    import torch

    import oracle
    import paper_2201_00094_amd as wt
    import synth

    smoke = args.workload == "smoke"
    t0 = time.perf_counter()
    f = synth.frame_c2(seed=args.seed, rank=args.rank) if smoke else synth.frame_c3(seed=args.seed, rank=args.rank)
    print("precision: generated %s, %d fragments in %.1f s" % (f.name, f.count, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    if args.sample_pixels <= 0 or args.sample_pixels >= f.pixels:
        sel, mask = np.arange(f.pixels), None
    else:
        rng = np.random.default_rng(args.seed + 5)
        sel = np.unique(rng.choice(f.pixels, args.sample_pixels, replace=False))
        mask = np.zeros(f.pixels, bool)
        mask[sel] = True
    C = f.channels
    t0 = time.perf_counter()
    ex = oracle.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=C, mask=mask,
                        want=("out",), tight=args.tight)["out"][sel]
    ab = oracle.abuffer(f.width, f.height, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=C, mask=mask)["out"][sel]
    print("precision: oracle and A-buffer on %d pixels in %.1f s" % (sel.size, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)

    def err(a, b):
        e = np.abs(a - b)
        return {"max": float(e.max()), "mean": float(e.mean()), "p99": float(np.percentile(e, 99))}

    res = {}
    ref32 = None
    for dt in (("f32", "f16", "bf16") if smoke else ("f32", "f16", "bf16", "e5b9g9r9")):
        spec = wt.FrameSpec(f.width, f.height, f.rank, C, dt, args.tight)
        ws = wt.Workspace(spec, f.count)
        coeffs = spec.new_coeffs()
        out = torch.empty((spec.pixels, 3), dtype=torch.float32, device="cuda")
        for _ in range(2):
            wt.render(spec, fr, f.bg, ws, out=out, coeffs=coeffs)
        torch.cuda.synchronize()
        K = max(1, args.steps // 2)
        t1 = time.perf_counter()
        for _ in range(K):
            wt.render(spec, fr, f.bg, ws, out=out, coeffs=coeffs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / K
        g = out.cpu().double().numpy()[sel]
        if dt == "f32":
            ref32 = g
        res[dt] = {"ms_per_frame": ms, "fragments_per_s": f.count / (ms * 1e-3),
                   "coeff_bytes_per_px": int(coeffs.element_size() * coeffs[0].numel()),
                   "vs_oracle_exact": err(g, ex), "vs_abuffer": err(g, ab), "vs_f32_storage": err(g, ref32)}
        print("precision: %s %.3f ms/frame, max |out - oracle| %.2e" % (dt, ms, res[dt]["vs_oracle_exact"]["max"]),
              file=sys.stderr, flush=True)
        del ws, coeffs, out
        torch.cuda.empty_cache()
    line = {"metric": "%s resolve: ms/frame and composite error per coefficient storage" % ("smoke" if smoke else
                                                                                            "glass + particles"),
            "mode": "precision", "n_gpus": 1, "data": "synthetic", "fragments": f.count,
            "pixels_checked": int(sel.size), "tight": bool(args.tight),
            "oracle_exact_vs_abuffer": err(ex, ab), "storage": res,
            "config": {"workload": ("smoke %dx%d, Poisson(64 g) fragments/px, rank %d, one visibility channel" %
                                    (f.width, f.height, f.rank)) if smoke else
                                   ("glass + particles %dx%d, 2-4 glass layers (per-channel alpha) + Poisson(24) "
                                    "particles per px, rank %d, three visibility channels" % (f.width, f.height,
                                                                                              f.rank))}}
    print(json.dumps(line))


def run_copy(args):
    """A plain 1 GiB device-to-device copy, repeated: the reference for scaling the FETCH_SIZE / WRITE_SIZE
    counters of the path's kernels to HBM bytes."""
    import torch
    n = 1 << 28  # floats: 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(args.steps, 1)):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read": n * 4, "bytes_written": n * 4, "copies": max(args.steps, 1)}))


def _counter_means(folder):
    """Mean counter value (KiB per dispatch) per demangled kernel name in a rocprofv3 --pmc csv folder."""
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % folder)
    acc = {}
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def run_traffic(args):
    """FETCH_SIZE and WRITE_SIZE per dispatch of the path's kernels, each scaled by what the same counter reads
    for the 1 GiB copy (bytes moved / counter KiB), written to the traffic summary with the kernel sources'
    digest."""
    fetch, write, cfetch, cwrite = (_counter_means(d) for d in args.pmc)
    copy_name = [k for k in cfetch if "copyBuffer" in k][0]
    gib = float(1 << 30)
    f_scale = gib / (cfetch[copy_name][0] * 1024.0)
    w_scale = gib / (cwrite[copy_name][0] * 1024.0)
    key = workload_key(args)
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        if t.get("sources_sha256") != sources_digest():
            t = {}
    except (OSError, ValueError):
        t = {}
    t["sources_sha256"] = sources_digest()
    t["fetch_scale"], t["write_scale"] = f_scale, w_scale
    t.setdefault("workloads", {})[key] = {}
    t.setdefault("commands", {})[key] = args.pmc_command
    rows = []
    for short, prefix in KERNEL_PREFIX.items():
        names = [k for k in fetch if k.startswith(prefix)]
        if not names:
            continue
        fk, n = fetch[names[0]]
        wk = write[names[0]][0]
        by = fk * 1024.0 * f_scale + wk * 1024.0 * w_scale
        t["workloads"][key][short] = by
        rows.append("| `%s` | %d | %.0f | %.0f | %.4g |" % (names[0].split("(")[0], n, fk, wk, by / 1e9))
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
    md = TRAFFIC_FILE[:-5] + "_%s.md" % key
    with open(md, "w") as fh:
        fh.write("# HBM traffic per launch, smoke 1920x1080, Poisson(64 g) fragments/px, rank %d, %s coefficients%s\n\n"
                 % (args.rank, args.dtype, (", per-pixel depth bounds" if args.tight else "") +
                    (", one pass against the previous frame" if args.temporal else "")))
        fh.write("Counters: rocprofv3 `--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`, in separate runs (KiB per dispatch, "
                 "mean over dispatches). Scale: a 1 GiB device copy (`bench.py --mode copy`) reads FETCH_SIZE "
                 "%.0f KiB and WRITE_SIZE %.0f KiB, so FETCH_SIZE is multiplied by %.4f and WRITE_SIZE by %.4f "
                 "(bytes per KiB counted / 1024).\n\n" % (cfetch[copy_name][0], cwrite[copy_name][0], f_scale,
                                                            w_scale))
        fh.write("Command (per counter, from /tmp with TMPDIR=/tmp):\n\n    %s\n\n" % args.pmc_command)
        fh.write("| Kernel | Dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM traffic (GB) |\n"
                 "| --- | --- | --- | --- | --- |\n")
        fh.write("\n".join(rows) + "\n")
    print(json.dumps(t["workloads"][key]))


def run_overlap(args):
    """Device overlap of the serving slots from a rocprofv3 kernel trace (``--trace``: the kernel_trace.csv of a
    ``--mode serve`` run): kernels grouped by HIP stream; a sweep over their start/end times gives the time any
    kernel runs, the time kernels of two or more streams run together, and how many kernels overlap a kernel of
    another stream."""
    rows = []
    with open(args.trace) as fh:
        for r in csv.DictReader(fh):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            name = r["Kernel_Name"]
            if not name.startswith(("void wt::", "wt::")):
                continue  # library kernels only (the trace also holds torch's set-up kernels)
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), int(r["Stream_Id"]), name))
    rows.sort()
    events = sorted([(b, 1, s) for b, e, s, _ in rows] + [(e, -1, s) for b, e, s, _ in rows])
    active = collections.Counter()
    busy = multi = 0
    last = events[0][0] if events else 0
    peak = 0
    for t, d, s in events:
        n_streams = sum(1 for v in active.values() if v > 0)
        if n_streams >= 1:
            busy += t - last
        if n_streams >= 2:
            multi += t - last
        active[s] += d
        peak = max(peak, sum(1 for v in active.values() if v > 0))
        last = t
    # kernels that run at the same time as at least one kernel of another stream (every overlapping pair has one
    # kernel starting inside the other, so a scan forward from each start-sorted kernel finds it)
    hit = [False] * len(rows)
    for i, (b, e, s, _) in enumerate(rows):
        for j in range(i + 1, len(rows)):
            if rows[j][0] >= e:
                break
            if rows[j][2] != s:
                hit[i] = hit[j] = True
    overlapped = sum(hit)
    streams = sorted({r[2] for r in rows})
    span = (max(e for _, e, _, _ in rows) - rows[0][0]) if rows else 0
    res = {"kernels": len(rows), "streams": len(streams), "span_ms": span * 1e-6, "busy_ms": busy * 1e-6,
           "two_or_more_streams_ms": multi * 1e-6, "share_of_busy_time_with_overlap": multi / busy if busy else 0.0,
           "max_streams_at_once": peak, "kernels_overlapping_another_streams_kernel": overlapped}
    print(json.dumps(res))


def run_serve(args):
    """Poisson arrivals of frames whose size is drawn from 640x360 .. 3840x2160, rank from {3, 4} and storage from
    {f32, f16}, 24 fragments/px; admitted by HBM footprint into a fixed number of slots; p50/p99 latency from
    arrival to completion, arrival-to-admission waits and whole-trace fragments/s, for a sweep of arrival rates
    (shares of the solo capacity). Every request is re-rendered alone afterwards and compared with its served
    result."""
    import torch

    import paper_2201_00094_amd as wt
    import synth
    from paper_2201_00094_amd.serve import FrameRequest, GpuExecutor, Server

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pool = {}
    for (w, h) in synth.REQUEST_RESOLUTIONS:
        for s in range(2):
            pix, dep, al, rgb = synth.torch_frame(1000 * s + w, w, h, mean=24.0, device=dev)
            pool[(w, h, s)] = wt.Fragments(pix, dep, al, rgb)
    torch.cuda.synchronize()
    # solo service time per (size, rank, storage), warm
    solo = {}
    for (w, h, s), fr in pool.items():
        if s:
            continue
        for rank in (3, 4):
            for dt in ("f32", "f16"):
                spec = wt.FrameSpec(w, h, rank, 1, dt)
                ws = wt.Workspace(spec, fr.count, device=dev)
                for _ in range(2):
                    wt.render(spec, fr, (0.2, 0.2, 0.2), ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    wt.render(spec, fr, (0.2, 0.2, 0.2), ws)
                torch.cuda.synchronize()
                solo[(w, h, rank, dt)] = (time.perf_counter() - t0) / 3
                del ws
    torch.cuda.empty_cache()
    mean_service = float(np.mean(list(solo.values())))
    sweep = []
    for k, load in enumerate(float(v) for v in str(args.load).split(",")):
        rate = load / mean_service
        trace = synth.poisson_arrivals(args.seed + k, args.requests, rate)
        ex = GpuExecutor(slots=args.slots, device=dev)
        # the slots' resident buffers sized for the largest request, and every request's composite buffer, before
        # the trace starts: no allocation while it runs
        big_w, big_h = max(synth.REQUEST_RESOLUTIONS, key=lambda wh: wh[0] * wh[1])
        ex.reserve(big_w, big_h, 4, max(q.count for kk, q in pool.items() if kk[:2] == (big_w, big_h)))
        outs = [torch.empty((r["width"] * r["height"], 3), dtype=torch.float32, device=dev) for r in trace]
        torch.cuda.synchronize()
        srv = Server(ex, slots=args.slots, budget_bytes=int(args.budget_gb * (1 << 30)), policy=args.policy)
        futs = []
        late = np.zeros(len(trace))
        t0 = time.perf_counter()
        for i, r in enumerate(trace):
            now = time.perf_counter() - t0
            if r["t"] > now:
                time.sleep(r["t"] - now)
            late[i] = time.perf_counter() - t0 - r["t"]  # how far the submission fell behind the trace
            fr = pool[(r["width"], r["height"], r["seed"] % 2)]
            futs.append(srv.submit(FrameRequest(r["width"], r["height"], r["rank"], fr, dtype=r["dtype"],
                                                bg=(0.2, 0.2, 0.2), tag=i, out=outs[i])))
        results = [fu.result(timeout=600) for fu in futs]
        srv.close()
        stats = srv.stats.summary()
        # latency from the trace's arrival times (the server's own figures start at submit)
        from_arrival = np.array([(res.t_done - t0 - r["t"]) * 1e3 for res, r in zip(results, trace)])
        # every request against the same frame rendered alone
        worst = 0.0
        alone_ws = {}
        for i, r in enumerate(trace):
            fr = pool[(r["width"], r["height"], r["seed"] % 2)]
            spec = wt.FrameSpec(r["width"], r["height"], r["rank"], 1, r["dtype"])
            key = (r["width"], r["height"], r["rank"], r["dtype"])
            if key not in alone_ws:
                most = max(q.count for kk, q in pool.items() if kk[:2] == (r["width"], r["height"]))
                alone_ws[key] = wt.Workspace(spec, most, device=dev)
            alone = wt.render(spec, fr, (0.2, 0.2, 0.2), alone_ws[key])
            worst = max(worst, float((alone - results[i].out).abs().max()))
        del alone_ws, results, ex, outs
        torch.cuda.empty_cache()
        sweep.append({"load": load, "rate_hz": rate, "requests": len(trace), "fragments_per_s": stats["fragments_per_s"],
                      "p50_ms": stats["p50_ms"], "p99_ms": stats["p99_ms"], "mean_ms": stats["mean_ms"],
                      "queued": stats["queued"], "wait_p50_ms": stats["wait_p50_ms"],
                      "wait_p99_ms": stats["wait_p99_ms"], "admitted": stats["completed"],
                      "rejected": stats["rejected"], "max_inflight": stats["max_inflight"],
                      "max_gb_inflight": stats["max_bytes_inflight"] / (1 << 30), "solo_vs_mix_max_abs": worst,
                      "arrival_p50_ms": float(np.percentile(from_arrival, 50)),
                      "arrival_p99_ms": float(np.percentile(from_arrival, 99)),
                      "submit_late_p99_ms": float(np.percentile(late, 99) * 1e3),
                      "submit_late_max_ms": float(late.max() * 1e3)})
        print("serve: load %.2f p50 %.2f ms p99 %.2f ms %.3g fragments/s; from arrival p50 %.2f p99 %.2f ms, "
              "submissions late by %.2f ms at p99" % (load, stats["p50_ms"], stats["p99_ms"], stats["fragments_per_s"],
                                                      sweep[-1]["arrival_p50_ms"], sweep[-1]["arrival_p99_ms"],
                                                      sweep[-1]["submit_late_p99_ms"]),
              file=sys.stderr, flush=True)
    head = sweep[min(1, len(sweep) - 1)]
    line = {"metric": "served frames: p50/p99 latency (arrival to completion) and fragments/s", "mode": "serve",
            "value": head["fragments_per_s"], "unit": "fragments/s", "n_gpus": 1, "load": head["load"],
            "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "mean_solo_ms": mean_service * 1e3,
            "slots": args.slots, "budget_gb": args.budget_gb, "policy": args.policy, "sweep": sweep,
            "solo_vs_mix_max_abs": max(x["solo_vs_mix_max_abs"] for x in sweep),
            "data": "synthetic", "dtype": "f32/f16 storage mix",
            "config": {"workload": "Poisson arrivals; 640x360..3840x2160, rank 3/4, f32/f16 storage, "
                                   "Poisson(24) fragments/px"}}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
