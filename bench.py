#!/usr/bin/env python3
"""Benchmark of the GridShift hot path on one MI355X.

Workload: the plain fit of a synthetic 1920x1080 Voronoi image (40 regions,
colour ramps, noise sigma 6) with features (0.25x, 0.25y, L*, a*, b*) as
float32 (d = 5, n = 2,073,600), h = 16, at most 100 rounds.  Inputs are
resident in HBM before the timed region; one step is one complete gs_fit
(binning, every shift/merge round, labels) plus the mode copy.

Prints one JSON line with points/s, the roofline of the dominant kernel
(algorithmic bytes per launch over its HIP-event-timed average duration) and
the FP64 oracle timed on the host cores as the CPU baseline.  The same line
carries, under "forms", the other two forms of the workload family:
  batched  256 Voronoi images of uneven size (heights 240..1080, widths
           320..1920, 5..60 regions, noise 4..12), RGB float32, per-image
           h in {12, 16, 24}, one gs_fit_batched call;
  fwd_bwd  64 Voronoi images of 512x512, (x, y, L, a, b) float32, h = 16:
           the point-to-mode loss and its gradient (fit with checkpoints
           every 8 tail rounds, loss, backward with segment recomputation);
  gmm      Gaussian mixtures of 10^7 float32 points, 50 components, h = 4,
           d = 2..6: the cost of the 3^d neighbour gather per dimension.
The plain form also reports its time per phase (binning, rounds, labels).

  python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--forms plain,batched,fwd_bwd,gmm,sequential,hsweep,track]
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/sec + HBM GB/s: GridShift 1080p d=5 plain vs batched vs fwd+bwd"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


@contextlib.contextmanager
def gc_paused():
    """Python's cyclic garbage collector held off over a timed region, as
    timeit does: a full collection of this process's objects (torch's among
    them) takes about 60 ms on the host and would otherwise land inside
    whichever step crosses its allocation threshold."""
    was = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def _profile_values(name: str):
    """key=value lines of a committed rocprofv3 summary under profiles/, or None
    when there is none or the sources it names changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    h = hashlib.sha256()
    for src in kv.get("sources", "").split(","):
        f = os.path.join(ROOT, "paper_2206_02200_amd", src)
        if not src or not os.path.exists(f):
            return None
        h.update(open(f, "rb").read())
    if h.hexdigest() != kv.get("sources_sha256"):
        return None
    return kv


def measured_traffic(kernel: str, workload: str = "plain_1080p_d5"):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE / WRITE_SIZE summary
    profiles/<kernel>_traffic_<workload>.txt, or None."""
    kv = _profile_values(f"{kernel}_traffic_{workload}.txt")
    return None if kv is None else float(kv["traffic_bytes_per_launch"])


def measured_counters(kernel: str, workload: str = "plain_1080p_d5"):
    """LDS and L2-atomic counters per launch of `kernel` from the summary
    profiles/lds_atomic_counters_<workload>.txt, or None."""
    kv = _profile_values(f"lds_atomic_counters_{workload}.txt")
    if kv is None or f"{kernel}.lds_insts" not in kv:
        return None
    fields = ("lds_insts", "lds_active_cycles", "lds_bank_conflict_cycles", "lds_conflict_ratio", "l2_atomics")
    return {f: float(kv[f"{kernel}.{f}"]) for f in fields}


def host_cores() -> int:
    """Host threads the instance-parallel oracle runs use: the CPUs this
    process may run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def form_roofline(ctx, run, reps: int, workload: str) -> dict:
    """Every kernel of `reps` untimed runs of a form timed with HIP events on
    its launch stream; the roofline object of the one with the largest total
    time (its algorithmic bytes per launch over its average launch time)."""
    import torch

    ctx.profile("")
    ctx.profile_reset()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    table = ctx.profile_table()
    ctx.profile(None)
    dom = max(table, key=lambda k: table[k]["ms"])
    e = table[dom]
    avg_ms = e["ms"] / e["launches"]
    bpl = e["bytes"] / e["launches"]
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    return {
        "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(dom, workload),
        "counters": measured_counters(dom, workload), "avg_launch_us": avg_ms * 1e3,
        "alg_bytes_per_launch": bpl, "launches_per_step": e["launches"] / reps,
        "kernels_ms_per_step": {k: v["ms"] / reps for k, v in sorted(table.items(), key=lambda t: -t[1]["ms"])},
    }


def oracle_instances(xs, hs, max_iter: int, cores: int, seconds: float):
    """The FP64 oracle on independent instances, one host thread per core
    (the oracle itself is single-threaded C; ctypes releases the GIL around
    it).  Runs instances in order until `seconds` have passed; returns
    (instances done, points done, wall seconds)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import gs_oracle

    gs_oracle.ensure_loaded()
    done = pts = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as pool:
        i = 0
        while i < len(xs) and (time.perf_counter() - t0) < seconds:
            chunk = list(range(i, min(len(xs), i + cores)))
            list(pool.map(lambda j: gs_oracle.fit(xs[j], float(hs[j]), max_iter), chunk))
            done += len(chunk)
            pts += sum(len(xs[j]) for j in chunk)
            i += len(chunk)
    return done, pts, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, seconds: float) -> dict:
    """The FP64 oracle (single-threaded C) on the same image, repeated for a
    bounded wall time."""
    import numpy as np

    from oracle import gs_oracle

    xd = w.x.astype(np.float64)
    runs = 0
    t0 = time.perf_counter()
    while True:
        gs_oracle.fit(xd, w.h, w.max_iter)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": runs * len(xd) / el,
        "unit": "points/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{runs} full fits of the same {len(xd)}-point image in {el:.1f} s "
                  f"(single thread; host: {os.cpu_count()} logical CPUs, {cpu_model()})",
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip every oracle timing (the headline baseline and those of the forms)")
    ap.add_argument("--form-cpu-seconds", type=float, default=8.0,
                    help="bound of each form's oracle timing (instances are started until it has passed)")
    ap.add_argument("--forms", default="plain,batched,fwd_bwd,gmm,sequential,hsweep,track")
    ap.add_argument("--form-only", choices=["batched", "fwd_bwd", "gmm", "sequential", "hsweep", "track"], default=None,
                    help="time only this form (--steps timed calls after one warm-up) and print its JSON object; "
                         "for profiling a form on its own")
    ap.add_argument("--gmm-d", default="2,3,4,5,6", help="dimensions of the Gaussian-mixture form")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched form: keep the default launch configuration (for counter runs, where the "
                         "tuner's fits would multiply the dispatches)")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="run an elementwise copy of this many MiB (read + write) before the fits, untimed: "
                         "the reference kernel that scales hardware byte counters taken on this command")
    args = ap.parse_args()
    forms = set(args.forms.split(","))
    if args.gpus != 1:
        print("bench.py measures one GPU only: the GridShift fit here runs on a single MI355X; "
              "run it with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2206_02200_amd import gridshift, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibration_copy_mb > 0:
        src = torch.ones(args.calibration_copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    gmm_dims = [int(v) for v in args.gmm_d.split(",")]
    if args.form_only:
        if args.form_only == "batched":
            res = bench_batched(gridshift.Context(0), dev, args.steps, 0.0, not args.no_autotune)
        elif args.form_only == "sequential":
            w = synth.image_xylab_f32()
            res = bench_sequential(torch.from_numpy(w.x).to(dev), w, args.steps)
        elif args.form_only == "hsweep":
            res = bench_hsweep(dev, args.steps)
        elif args.form_only == "track":
            res = bench_track(dev, args.steps)
        elif args.form_only == "gmm":
            res = bench_gmm(dev, args.steps, 0.0, gmm_dims)
        else:
            res = bench_fwd_bwd(dev, args.steps, 0.0)
        print(json.dumps(res), flush=True)
        return 0
    w = synth.image_xylab_f32()
    n, d = w.x.shape
    x = torch.from_numpy(w.x).to(dev)
    ctx = gridshift.Context(0)

    def step():
        return gridshift.fit(x, w.h, w.max_iter, ctx=ctx)

    for _ in range(max(1, args.warmup)):
        r = step()
    torch.cuda.synchronize()
    info = r.info

    # every kernel timed over a few untimed steps: per-kernel split
    ctx.profile("")
    ctx.profile_reset()
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    full = ctx.profile_table()
    ctx.profile(None)
    dominant = max(full, key=lambda k: full[k]["ms"])

    # timed region: HIP events around the dominant kernel's launches only
    ctx.profile_reset()
    ctx.profile(dominant)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ctx.profile(None)
    dom = ctx.profile_table()[dominant]

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3)
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    s_in = w.x.dtype.itemsize
    k = info["n_clusters"]
    # point-level algorithmic bytes of the whole fit: read x once, write and
    # read the point->cell map, write labels; plus the first round's cell table
    b_alg = n * (d * s_in + 12) + 2 * info["n_cells0"] * (16 + 8 * d) + k * (8 * d + 8)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain GridShift, 1920x1080 Voronoi image (40 regions, ramps, sigma 6), "
                        "features (0.25x, 0.25y, L, a, b) float32, d=5, h=16, max_iter=100",
            "n": n, "d": d, "h": w.h, "max_iter": w.max_iter, "input_dtype": "f32",
            "cells0": info["n_cells0"], "clusters": k, "rounds": info["n_iter"], "flags": info["flags"],
        },
        "hbm_GBps_step_alg": b_alg / (ms_per_step * 1e-3) / 1e9,
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": measured_traffic(dominant),
            "counters": measured_counters(dominant),
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": bytes_per_launch,
        },
        "kernels_ms_per_step": {kk: vv["ms"] / 3 for kk, vv in sorted(full.items(), key=lambda t: -t[1]["ms"])},
        "phases_ms_per_step": phase_split(full, 3),
    }
    out["forms"] = {"plain": {"value": value, "unit": "points/s", "ms_per_step": ms_per_step,
                              "hbm_GBps_alg": out["hbm_GBps_step_alg"]}}
    cpu_s = 0.0 if args.no_cpu_baseline else args.form_cpu_seconds
    out["forms"]["plain"]["result_api"] = bench_result_api(x, w, args.steps, ms_per_step)
    if "batched" in forms:
        out["forms"]["batched"] = bench_batched(ctx, dev, max(5, args.steps // 4), cpu_s, not args.no_autotune)
    if "sequential" in forms:
        out["forms"]["sequential"] = bench_sequential(x, w, max(1, args.steps // 2))
    if "gmm" in forms:
        out["forms"]["gmm"] = bench_gmm(dev, max(1, args.steps // 4), cpu_s, gmm_dims)
    if "hsweep" in forms:
        out["forms"]["hsweep"] = bench_hsweep(dev, max(1, args.steps // 4))
    if "track" in forms:
        out["forms"]["track"] = bench_track(dev, max(1, args.steps // 10))
    if "fwd_bwd" in forms:
        out["forms"]["fwd_bwd"] = bench_fwd_bwd(dev, max(5, args.steps // 4), cpu_s)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


# Kernels of the binning phase of a plain fit (its single device-wide merge
# runs in one workgroup, so every sort pass and heads scan belongs to the
# binning); the labels kernel is its own phase; everything else is rounds.
BIN_KERNELS = ("bbox", "make_keys", "sort_pass", "scan_heads", "bin_cell_setup", "bin_scan_chunks",
               "bin_segsum_chunks", "bin_segsum_levels")


def phase_split(table: dict, fits: int) -> dict:
    out = {"binning": 0.0, "rounds": 0.0, "labels": 0.0}
    for name, v in table.items():
        ph = "binning" if name in BIN_KERNELS else ("labels" if name == "labels" else "rounds")
        out[ph] += v["ms"] / fits
    return out


def bench_sequential(x, w, steps: int) -> dict:
    """The same 1080p fit with the sequential update of Eq. 5 (swept colour by
    colour): throughput, and the rounds and clusters it takes."""
    import torch

    from paper_2206_02200_amd import gridshift

    ctx = gridshift.Context(0)
    ctx.set_update("sequential")
    r = gridshift.fit(x, w.h, w.max_iter, ctx=ctx)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            r = gridshift.fit(x, w.h, w.max_iter, ctx=ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    n = x.shape[0]
    out = {"value": n / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "steps": steps,
           "rounds": r.info["n_iter"], "clusters": r.info["n_clusters"], "flags": r.info["flags"],
           "workload": "plain 1920x1080 (0.25x, 0.25y, L, a, b) f32, d=5, h=16, update of Eq. 5 by colours"}
    ctx.close()
    return out


def bench_hsweep(dev, steps: int) -> dict:
    """Bandwidth sweep: 1e6 points of a clustering set scaled into [0,1]^3,
    fitted at h = 0.02, 0.04, ..., 1.00 (50 values) in one batched pass."""
    import torch

    from paper_2206_02200_amd import gridshift, synth

    n, d = 1_000_000, 3
    x = torch.from_numpy(synth.unit_gmm_f32(n, d, seed=95)).to(dev)
    hs = synth.hsweep_grid(50)
    ctx = gridshift.Context(0)
    r = gridshift.fit_hsweep(x, hs, 100, ctx=ctx)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            r = gridshift.fit_hsweep(x, hs, 100, ctx=ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {"value": n * len(hs) / (ms * 1e-3), "unit": "points/s (points x bandwidths)", "ms_per_step": ms,
           "steps": steps, "n": n, "d": d, "bandwidths": len(hs),
           "clusters_by_h": {f"{h:.2f}": i["n_clusters"] for h, i in zip(hs, r.infos)},
           "rounds_by_h": {f"{h:.2f}": i["n_iter"] for h, i in zip(hs, r.infos)},
           "workload": "1e6 points, 12-component Gaussian mixture scaled into [0,1]^3, f32, "
                       "h = 0.02..1.00 step 0.02, one batched pass"}
    ctx.close()
    return out


def bench_track(dev, steps: int) -> dict:
    """Object tracking (Algorithm 2): a 640x480 RGB float32 video of 200
    frames, one moving disc; the whole sequence (initial GridShift + every
    frame) per step."""
    import numpy as np
    import torch

    from paper_2206_02200_amd import gridshift, synth

    frames, centres = synth.moving_blob_video(T=200, H=480, W=640, radius=28.0, seed=7)
    fr = torch.from_numpy(frames).to(dev)
    ctx = gridshift.Context(0)
    args = (fr, centres[0], 48.0, 48.0, 0.8, 16.0, 0.5, 20)
    win = gridshift.track(*args, ctx=ctx)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            win = gridshift.track(*args, ctx=ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    T = frames.shape[0]
    out = {"value": T / (ms * 1e-3), "unit": "frames/s", "ms_per_step": ms, "steps": steps, "frames": T,
           "max_centre_error_px": float(np.abs(win[:, :2] - centres).max()),
           "workload": "640x480 RGB f32, 200 frames, one textured disc (radius 28) moving 2-5 px/frame; "
                       "h=16, f=0.8, eta=0.5, max_inner=20, the largest initial cluster"}
    # many objects at once: 32 discs (radius 14), one workgroup per track
    nd = 32
    frames, centres = synth.moving_blob_video(T=200, H=480, W=640, radius=14.0, seed=8, discs=nd)
    fr = torch.from_numpy(frames).to(dev)
    bargs = (fr, centres[0], np.full(nd, 24.0), np.full(nd, 24.0), 0.8, 16.0, 0.5, 20)
    bw = gridshift.track_batched(*bargs, ctx=ctx)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            bw = gridshift.track_batched(*bargs, ctx=ctx)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t0) * 1e3 / steps
    err = np.abs(bw[:, :, :2] - np.transpose(centres, (1, 0, 2)))
    out["batched"] = {"value": nd * T / (bms * 1e-3), "unit": "track-frames/s", "ms_per_step": bms, "tracks": nd,
                      "median_centre_error_px": float(np.median(err)),
                      "workload": "640x480 RGB f32, 200 frames, 32 textured discs (radius 14) of distinct colours, "
                                  "one track each, one launch"}
    ctx.close()
    return out


def bench_gmm(dev, steps: int, cpu_seconds: float, dims=(2, 3, 4, 5, 6)) -> dict:
    """Gaussian mixtures of 1e7 float32 points, d = 2..6: the 3^d neighbour
    probes of the device-wide rounds, as probes/s of the shift kernel, and
    the dominant kernel per d."""
    import numpy as np
    import torch

    from paper_2206_02200_amd import gridshift, synth

    ctx = gridshift.Context(0)
    res = {}
    for d in dims:
        w = synth.gmm_f32(10_000_000, d, seed=40 + d)
        x = torch.from_numpy(w.x).to(dev)
        n = w.x.shape[0]
        r = gridshift.fit(x, w.h, w.max_iter, ctx=ctx)  # warm-up (allocations)
        torch.cuda.synchronize()
        with gc_paused():
            t0 = time.perf_counter()
            for _ in range(steps):
                r = gridshift.fit(x, w.h, w.max_iter, ctx=ctx)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
        info = r.info
        m0, k = info["n_cells0"], info["n_clusters"]
        b_alg = n * (d * 4 + 12) + 2 * m0 * (16 + 8 * d) + k * (8 * d + 8)
        roof = form_roofline(ctx, lambda: gridshift.fit(x, w.h, w.max_iter, ctx=ctx), 2, f"gmm_1e7_d{d}")
        sh_ms = roof["kernels_ms_per_step"].get("shift", 0.0)
        # the shift's algorithmic bytes are (28 + 16d) per cell of its round:
        # the cells it moved, each probing its 3^d neighbour keys
        ctx.profile("shift")
        ctx.profile_reset()
        gridshift.fit(x, w.h, w.max_iter, ctx=ctx)
        torch.cuda.synchronize()
        sh = ctx.profile_table().get("shift", {"ms": 0.0, "launches": 0, "bytes": 0.0})
        ctx.profile(None)
        shift_cells = sh["bytes"] / (28.0 + 16.0 * d)
        probes = shift_cells * 3 ** d
        ent = {
            "value": n / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "steps": steps,
            "hbm_GBps_alg": b_alg / (ms * 1e-3) / 1e9, "cells0": m0, "clusters": k, "rounds": info["n_iter"],
            "shift_ms_per_fit": sh["ms"], "shift_launches": sh["launches"], "shift_cells": shift_cells,
            "neighbour_probes": probes, "probes_per_s": probes / (sh["ms"] * 1e-3) if sh["ms"] > 0 else None,
            "shift_ms_per_fit_profiled_run": sh_ms, "roofline": roof,
        }
        if cpu_seconds > 0:
            # the oracle (one thread) on a prefix of the same i.i.d. points
            from oracle import gs_oracle

            npre = 1_000_000
            xs = w.x[:npre].astype(np.float64)
            runs, t0 = 0, time.perf_counter()
            while True:
                gs_oracle.fit(xs, w.h, w.max_iter)
                runs += 1
                if time.perf_counter() - t0 >= cpu_seconds / 5:
                    break
            el = time.perf_counter() - t0
            ent["cpu_baseline"] = {"value": runs * npre / el, "unit": "points/s", "cores": 1, "kind": "oracle",
                                   "sample": f"{runs} fits of the first {npre} points of the same mixture "
                                             f"in {el:.1f} s (single thread)"}
        res[f"d{d}"] = ent
        del x
    ctx.close()
    res["workload"] = ("Gaussian mixture, 50 isotropic components, means U[0,100]^d, sigma U[1,3], "
                       "Dirichlet(1) weights, n=1e7 f32, h=4, max_iter=100")
    return res


def bench_batched(ctx, dev, steps: int, cpu_seconds: float, tune: bool = True) -> dict:
    import numpy as np
    import torch

    from paper_2206_02200_amd import gridshift, synth

    specs = synth.batch_specs()
    X, off, hs = synth.batch_rgb_torch(specs, dev)
    n = int(off[-1])
    r = gridshift.fit_batched(X, off, hs, 100, ctx=ctx)  # warm-up (allocations)
    torch.cuda.synchronize()
    # the launch configuration: every candidate timed on this batch, the fastest kept
    t_tune = t_cached = None
    cfg = ctx.config()
    if tune:
        t_tune = time.perf_counter()
        cfg = ctx.autotune(X, hs, 100, offsets=off, reps=1)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t_tune
        # the same shape again: the choice comes from the cache, no fit runs
        t_cached = time.perf_counter()
        ctx.autotune(X, hs, 100, offsets=off, reps=1)
        t_cached = time.perf_counter() - t_cached
    # warm-up of the chosen configuration: two fits, so that torch's caching
    # allocator holds the output blocks of two results alive at once (the
    # previous result lives until the next call returns)
    for _ in range(2):
        r = gridshift.fit_batched(X, off, hs, 100, ctx=ctx)
    torch.cuda.synchronize()
    # each step timed on its own; the median is reported (a single step held
    # up by the host would otherwise dominate the few steps of this form)
    with gc_paused():
        step_ms = []
        for _ in range(steps):
            t0 = time.perf_counter()
            r = gridshift.fit_batched(X, off, hs, 100, ctx=ctx)
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(step_ms))
    rounds = [i["n_iter"] for i in r.infos]
    cells0 = sum(i["n_cells0"] for i in r.infos)
    k = int(r.k_offsets[-1])
    b_alg = n * (3 * 4 + 12) + 2 * cells0 * (16 + 8 * 3) + k * (8 * 3 + 8)
    out = {
        "value": n / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "steps": steps,
        "step_ms": [round(t, 3) for t in step_ms],
        "workload": "256 Voronoi images, H 240..1080, W 320..1920, 5..60 regions, sigma 4..12, RGB f32, "
                    "h in {12,16,24}, max_iter=100, one batched call, launch configuration autotuned on the batch",
        "n": n, "B": len(specs), "cells0": cells0, "clusters": k, "rounds_max": max(rounds),
        "rounds_mean": float(np.mean(rounds)), "capped": int(sum(1 for i in r.infos if i["flags"] & 4)),
        "hbm_GBps_alg": b_alg / (ms * 1e-3) / 1e9,
        "launch_config": cfg, "autotune_s": t_tune, "autotune_cached_s": t_cached,
        "roofline": form_roofline(ctx, lambda: gridshift.fit_batched(X, off, hs, 100, ctx=ctx), 1,
                                  "batched_256_images"),
    }
    if cpu_seconds > 0:
        # the oracle on the same bytes, instance-parallel over the host cores
        Xh = X.cpu().numpy()
        xs = [Xh[off[b]:off[b + 1]] for b in range(len(specs))]
        cores = host_cores()
        done, pts, el = oracle_instances(xs, hs, 100, cores, cpu_seconds)
        out["cpu_baseline"] = {"value": pts / el, "unit": "points/s", "cores": cores, "kind": "oracle",
                               "sample": f"{done} of the {len(specs)} images ({pts} points) in {el:.1f} s, "
                                         f"one image per thread on {cores} threads ({cpu_model()})"}
    return out


def bench_fwd_bwd(dev, steps: int, cpu_seconds: float) -> dict:
    import numpy as np
    import torch

    from paper_2206_02200_amd import gridshift, synth

    B = 64
    X, off = synth.diff_batch_torch(B, dev)
    n = int(off[-1])
    gctx = gridshift.Context(0)
    x = X.clone().requires_grad_(True)

    def step():
        x.grad = None
        loss = gridshift.point_mode_loss(x, 16.0, 100, off, gctx, ckpt_every=8)
        loss.sum().backward()
        return loss

    for _ in range(2):  # warm-up (allocations of two live results)
        loss = step()
    torch.cuda.synchronize()
    with gc_paused():
        step_ms = []  # each step on its own, the median reported
        for _ in range(steps):
            t0 = time.perf_counter()
            loss = step()
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(step_ms))
    # points read twice (fit, loss) plus the backward's read of x, labels and cell map and its f64 write
    b_alg = n * (5 * 4 + 12) + n * (5 * 4 + 4) + n * (4 + 5 * 4 + 4 + 8 * 5)
    out = {
        "value": n / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "steps": steps,
        "step_ms": [round(t, 3) for t in step_ms],
        "workload": "64 Voronoi images 512x512, 30 regions, ramps, sigma 6, (x,y,L,a,b) f32, h=16, "
                    "point-to-mode loss forward + backward (tail checkpoints every 8 rounds, recomputed in the backward)",
        "n": n, "B": B, "loss_mean": float(loss.detach().mean()), "hbm_GBps_alg": b_alg / (ms * 1e-3) / 1e9,
        "roofline": form_roofline(gctx, step, 1, "fwd_bwd_64x512"),
    }
    if cpu_seconds > 0:
        # the oracle's loss and gradient (fit with the trajectory, the loss, the
        # adjoint), instance-parallel over the host cores
        from concurrent.futures import ThreadPoolExecutor

        from oracle import gs_oracle

        Xh = X.cpu().numpy()
        cores = host_cores()
        gs_oracle.ensure_loaded()
        done = pts = 0
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=cores) as pool:
            while done < B and time.perf_counter() - t0 < cpu_seconds:
                chunk = list(range(done, min(B, done + cores)))
                list(pool.map(lambda j: gs_oracle.loss_and_grad(Xh[off[j]:off[j + 1]], 16.0, 100), chunk))
                done += len(chunk)
                pts += sum(int(off[j + 1] - off[j]) for j in chunk)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": pts / el, "unit": "points/s", "cores": cores, "kind": "oracle",
                               "sample": f"loss + gradient of {done} of the {B} images ({pts} points) in "
                                         f"{el:.1f} s, one image per thread on {cores} threads ({cpu_model()})"}
    gctx.close()
    return out


def bench_result_api(x, w, steps: int, ctx_ms: float) -> dict:
    """The boundary call itself: gs_fit with torch's caching allocator (a new
    result per fit), the mode copy and gs_result_free, per step, beside the
    same fit on a kept context."""
    import torch

    from paper_2206_02200_amd import gridshift

    def step():
        r = gridshift.fit_result(x, w.h, w.max_iter, allocator="torch")
        r.copy()
        r.close()

    step()
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_step": ms, "value": x.shape[0] / (ms * 1e-3), "unit": "points/s", "steps": steps,
            "vs_context_fit": ms / ctx_ms,
            "workload": "the plain workload through gs_fit + gs_result_copy + gs_result_free, device memory "
                        "from torch's caching allocator"}


if __name__ == "__main__":
    sys.exit(main())
