#!/usr/bin/env python3
"""Throughput of the off-axis holography path on one MI355X.

One step = dh_process_batch over a batch of 1000 synthetic 640x512 float32
frames, two polarisations (320x512 windows), HG groups G=9 (45 modes per
pol), FP32 path: row FFT -> column FFT + window crop + IFFT along y ->
IFFT along x + tilt/defocus removal + HG overlap -> FP64 power norm. Frames
are resident in HBM before the timed region. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import dh_synth  # noqa: E402

METRIC = "frames/s (FFT→IFFT→HG coefs) 640×512 maxMG=9, vs FP32 plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def stage_bytes(info, params, frames):
    """Algorithmic bytes per launch stage for `frames` frames: what each
    kernel must read and write (frame window in, its result out)."""
    P = params["pol_count"]
    nx, ny, wx, wy = info.fft_w, info.fft_h, info.ifft_w, info.ifft_h
    bx = info.box_w
    px = 2 if params.get("input_dtype", "f32") == "u16" else 4
    nm = info.modes
    return {
        "fft_x": frames * P * ny * (nx * px + bx * 8),
        "fft_y_crop_ifft_y": frames * P * bx * 8 * (ny + wy),
        "ifft_x_tilt_overlap": frames * P * (wy * bx * 8 + nm * 8),
        "power_norm": frames * P * nm * 16,
    }


STAGE_KERNEL = {"fft_x": "dh::k_row", "fft_y_crop_ifft_y": "dh::k_col", "ifft_x_tilt_overlap": "dh::k_fld",
                "power_norm": "dh::k_norm"}


def counter_traffic(stage, frames_per_launch):
    """HBM bytes per launch of `stage`'s kernel from the committed counter
    summary (profiles/traffic_c2_640x512.json), or None if the kernel sources
    changed since the counters were taken."""
    path = os.path.join(HERE, "profiles", "traffic_c2_640x512.json")
    if not os.path.exists(path):
        return None
    import bench_traffic
    t = json.load(open(path))
    if t.get("fingerprint") != bench_traffic.source_fingerprint():
        return None
    for name, k in t["kernels"].items():
        if name.startswith(STAGE_KERNEL[stage]):
            return round((k["read_bytes_per_frame"] + k["write_bytes_per_frame"]) * frames_per_launch)
    return None


def time_forms(dh, torch, cfg, ft, B, stream, steps=10, warmup=3):
    """frames/s and overlap-kernel time of the three overlap forms (plain FP32,
    split BF16, split FP16) on the same frames, at G=9 and G=20."""
    out = {}
    for groups in (9, 20):
        for prec in ("fp32", "split_bf16", "split_fp16"):
            plan = dh.Plan(dict(cfg["params"], max_mg=groups, precision=prec), max_batch=B)
            for _ in range(warmup):
                plan.process(ft, B, stream)
            stream.synchronize()
            plan.set_stage_timing(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                plan.process(ft, B, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            st = plan.stage_times()
            plan.destroy()
            ms = e0.elapsed_time(e1)
            out[f"G{groups}_{prec}"] = {"frames_per_s": round(steps * B / (ms / 1e3), 1),
                                        "overlap_kernel_ms": round(st["ifft_x_tilt_overlap"][0] / steps, 4)}
    return out


def cpu_baseline(cfg, frames, seconds):
    """The FP64 oracle, as it stands, on a bounded sample of the same frames."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    p = cfg["params"]
    g = oracle.geometry(p)
    oracle.process_frame(frames[0].astype(np.float64), p, g)   # warm caches
    n = 0
    t0 = time.perf_counter()
    while n < frames.shape[0] and (n < 4 or time.perf_counter() - t0 < seconds):
        oracle.process_frame(frames[n].astype(np.float64), p, g)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} frames of the same batch, one at a time, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 / split BF16 / split FP16 comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of 512 MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 512 * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(frames shard with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)

    cfg = dh_synth.config(1)
    B = args.frames
    t0 = time.time()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    frames, _ = dh_synth.make_frames(cfg, n_frames=B, workers=workers)   # before any GPU use
    print(f"[bench] synthesised {B} frames in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch
    import paper_2204_02348_amd as dh

    dev = torch.device("cuda:0")
    ft = torch.from_numpy(frames).to(dev)
    plan = dh.Plan(cfg["params"], max_batch=B)
    info = plan.info
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        plan.process(ft, B, stream)
    stream.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    plan.set_stage_timing(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        starts[k].record(stream)
        plan.process(ft, B, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.set_stage_timing(False)
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    total_ms = starts[0].elapsed_time(ends[-1])
    value = args.steps * B / (total_ms / 1e3)
    print(f"[bench] timed {args.steps} steps: {total_ms:.2f} ms", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    sb = stage_bytes(info, cfg["params"], B)
    dom = max(stages, key=lambda k: stages[k][0])
    ms_dom, n_dom = stages[dom]
    per_launch_bytes = sb[dom] / (n_dom / args.steps)
    achieved = per_launch_bytes / (ms_dom / n_dom / 1e3) / 1e9
    frames_per_launch = B / (n_dom / args.steps)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counter_traffic(dom, frames_per_launch) if B == 1000 else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes": round(per_launch_bytes), "kernel": dom,
                "launch_ms": round(ms_dom / n_dom, 4), "launches_per_step": n_dom // args.steps}
    frame_bytes = frames[0].nbytes
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1000 frames 640x512 f32, 2 pols (320x512 windows), G=9 (45 modes/pol), "
                               "defocus, shot+read noise; plain FP32 path",
                   "frames": B, "frame": "640x512", "pols": 2, "max_mg": 9, "precision": "fp32"},
        "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "path_hbm_frac": round(frame_bytes * value / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
    }
    plan.destroy()
    if not args.no_forms:
        out["forms"] = time_forms(dh, torch, cfg, ft, B, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, frames, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
