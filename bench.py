#!/usr/bin/env python3
"""Throughput of the off-axis holography path on one MI355X.

One step = dh_process_batch over a batch of 1000 synthetic 640x512 float32
frames, two polarisations (320x512 windows), HG groups G=9 (45 modes per
pol), plain FP32: row FFT -> column FFT + window crop -> (field path) IFFT
along y, IFFT along x + tilt/defocus removal + HG overlap, or (spectral path,
the default here) the window contracted with the folded IFFT/tilt/HG tables
-> FP64 power norm. Frames are resident in HBM before the timed region.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
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


def col_cg(ny):
    """Box columns per column-pass workgroup (the library's rule)."""
    return 4 if ny >= 1024 else 8 if ny >= 512 else 16


def stage_bytes(info, params, frames):
    """Algorithmic bytes per launch stage for `frames` frames: what each
    kernel must read and write (its input once, its result once)."""
    P = params["pol_count"]
    nx, ny, wx, wy = info.fft_w, info.fft_h, info.ifft_w, info.ifft_h
    bx = info.box_w
    px = 2 if params.get("input_dtype", "f32") == "u16" else 4
    nm = info.modes
    spectral = info.path == 2
    nblk = -(-bx // col_cg(ny)) if spectral else -(-wy // 16)
    return {
        "row_fft": frames * P * ny * (nx * px + bx * 8),
        # t1 columns in; f2 rows out (field) or per-column-block partials out (spectral)
        "column_fft_window": frames * P * (bx * ny * 8 + (nblk * (nm + 1) * 8 if spectral else wy * bx * 8)),
        "field_overlap": 0 if spectral else frames * P * (wy * bx * 8 + nblk * (nm + 1) * 8),
        "power_norm": frames * P * (nblk + 2) * (nm + 1) * 8,
    }


def frame_bytes_of(params):
    px = 2 if params.get("input_dtype", "f32") == "u16" else 4
    return params["frame_w"] * params["frame_h"] * px


def algorithmic_bytes_per_frame(params, info):
    """The path's algorithmic HBM bytes per frame: the input frame read once
    plus the raw coefficients written once (complex64 per mode and pol)."""
    return frame_bytes_of(params) + params["pol_count"] * info.modes * 8


def nominal_mflop_per_frame(params, info):
    """Nominal arithmetic of the paper's pipeline per frame (MFLOP): the 2D
    real FFT of each pol window (2.5 N log2 N), the complex IFFT of the Fourier
    window (5 M log2 M), the tilt/defocus phase (6 flop per field value) and
    the separable overlap (4 Wy Wx G + 4 G^2 Wy)."""
    import math
    n = info.fft_w * info.fft_h
    m = info.ifft_w * info.ifft_h
    g = params["max_mg"]
    per_pol = (2.5 * n * math.log2(n) + 5 * m * math.log2(m) + 6 * m
               + 4 * info.ifft_h * info.ifft_w * g + 4 * g * g * info.ifft_h)
    return params["pol_count"] * per_pol / 1e6


FP32_VECTOR_PEAK_TFLOPS = 157.3      # packed (dual) FP32; plain FP32 FMA issue gives half


def config_fraction(name, params, info, frames_per_s, workload):
    """frames/s of one workload against the HBM ceiling (algorithmic bytes) and
    the FP32 vector ceiling (nominal flops); the lower ceiling binds."""
    ab = algorithmic_bytes_per_frame(params, info)
    mf = nominal_mflop_per_frame(params, info)
    hbm_ceiling = HBM_PEAK_GBS * 1e9 / ab
    alu_ceiling = FP32_VECTOR_PEAK_TFLOPS * 1e12 / (mf * 1e6)
    bound = "hbm" if hbm_ceiling <= alu_ceiling else "alu"
    return {"workload": workload, "frames_per_s": round(frames_per_s, 1),
            "algorithmic_bytes_per_frame": int(ab), "nominal_mflop_per_frame": round(mf, 2),
            "hbm_frac": round(frames_per_s * ab / (HBM_PEAK_GBS * 1e9), 4),
            "alu_frac": round(frames_per_s * mf * 1e6 / (FP32_VECTOR_PEAK_TFLOPS * 1e12), 4),
            "bound": bound, "ceiling_frames_per_s": round(min(hbm_ceiling, alu_ceiling), 1),
            "frac_of_ceiling": round(frames_per_s / min(hbm_ceiling, alu_ceiling), 4)}


def stage_kernel(stage, info):
    return {"row_fft": "dh::k_row", "column_fft_window": "dh::k_cspec" if info.path == 2 else "dh::k_col",
            "field_overlap": "dh::k_fld", "power_norm": "dh::k_norm"}[stage]


def counter_traffic(stage, info, frames_per_launch):
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
        if name.startswith(stage_kernel(stage, info)):
            return round((k["read_bytes_per_frame"] + k["write_bytes_per_frame"]) * frames_per_launch)
    return None


def warm(plan, ft, n, stream, min_steps, min_s=0.06):
    """Untimed steps until at least min_steps have run and min_s of wall time
    has passed: the VALU-bound column passes run slower until the engine
    clock has ramped under ~20 ms of sustained work, and a count of short
    steps alone can end inside that ramp."""
    t0 = time.perf_counter()
    k = 0
    while k < min_steps or time.perf_counter() - t0 < min_s:
        plan.process(ft, n, stream)
        k += 1
        if k % 8 == 0:
            stream.synchronize()
    stream.synchronize()


def time_forms(dh, torch, cfg, ft, B, stream, steps=20, warmup=20):
    """frames/s and per-stage time of the coefficient forms on the same frames,
    at G=9 and G=20: plain FP32 on the field path and (where it applies) on
    the spectral path, split BF16 and split FP16 (field path); and at G=9 IFFT
    mode 0 (coefficients alone, and with the full-size fields exported)."""
    out = {}
    for groups in (9, 20):
        forms = [("fp32", "field", 1, 0), ("fp32", "spectral", 1, 0), ("split_bf16", "field", 1, 0),
                 ("split_fp16", "field", 1, 0)]
        if groups == 9:
            forms += [("fp32", "spectral", 0, 0), ("fp32", "spectral", 0, 1)]
        for prec, path, mode, fields in forms:
            d = dict(cfg["params"], max_mg=groups, precision=prec, path=path, ifft_mode=mode, keep_fields=fields)
            if dh.plan_check(d, B)[0] != dh.SUCCESS:
                continue
            plan = dh.Plan(d, max_batch=B)
            warm(plan, ft, B, stream, warmup)
            # frames/s from a window without per-launch events, then the
            # stage times from a second window with them
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                plan.process(ft, B, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            plan.set_stage_timing(True)
            for _ in range(steps):
                plan.process(ft, B, stream)
            torch.cuda.synchronize()
            st = plan.stage_times()
            plan.destroy()
            name = f"G{groups}_{prec}_{path}" + ("" if mode else "_mode0") + ("_fields" if fields else "")
            out[name] = {
                "frames_per_s": round(steps * B / (ms / 1e3), 1),
                "stages_ms": {k: round(v[0] / steps, 4) for k, v in st.items() if v[1]}}
            if groups == 20 and prec == "fp32" and path == "spectral" and mode == 1:
                info = dh.plan_check(d, B)[1]
                out["_c3"] = config_fraction("c3", d, info, steps * B / (ms / 1e3),
                                             "1000 frames 640x512 f32, 2 pols, G=20 (210 modes/pol), FP32")
    return out


def time_variants(dh, torch, cfg, ft, B, stream, steps=20, warmup=10):
    """Input frames/s of the batch variants on the same 1000 frames (G=9,
    spectral path): a sweep of 4 wavelengths (fast in, slow out), averaging of
    4 frames per output (sequential), and LG coefficients."""
    out = {}
    lams = [cfg["params"]["wavelength"] * (1 + d) for d in (-0.006, -0.002, 0.002, 0.006)]
    for name in ("sweep4", "avg4", "lg"):
        plan = dh.Plan(cfg["params"], max_batch=B)
        n_out = B
        if name == "sweep4":
            plan.set_wavelengths(lams, dh.WL_FAST, dh.WL_SLOW)
        elif name == "avg4":
            plan.set_averaging(4, dh.AVG_SEQUENTIAL)
            n_out = B // 4
        else:
            plan.set_basis(dh.BASIS_LG)
        warm(plan, ft, n_out, stream, warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.process(ft, n_out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.destroy()
        out[name] = {"input_frames_per_s": round(steps * B / (e0.elapsed_time(e1) / 1e3), 1), "outputs": n_out}
    return out


def time_aux(dh, torch, cfg, ft, B, stream, reps=20):
    """The kernels around the path on the benchmark batch: the int16 field
    conversion (HBM bound: 8 B read + 4 B written per field value) and the
    nine transfer-matrix metrics of the 1000 x 90 matrix (FP64 Gram,
    Jacobi eigenvalues, one host sync)."""
    out = {}
    plan = dh.Plan(dict(cfg["params"], keep_fields=1), max_batch=B)
    plan.process(ft, B, stream)
    stream.synchronize()
    nf = B * cfg["params"]["pol_count"]
    info = plan.info
    flen = info.field_w * info.field_h
    dev = ctypes.c_void_p()                # the plan's own device field buffer
    if dh.lib().dh_get_fields(plan.handle, None, ctypes.byref(dev), None, None, None, None) != dh.SUCCESS:
        raise RuntimeError("dh_get_fields")
    fields = dev.value
    re = torch.empty((nf, flen), dtype=torch.int16, device="cuda:0")
    im = torch.empty_like(re)
    sc = torch.empty(nf, dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        dh.fields_to_int16(fields, nf, flen, re, im, sc, stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dh.fields_to_int16(fields, nf, flen, re, im, sc, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = nf * flen * 12 / (ms * 1e-3) / 1e9
    out["int16_fields"] = {"fields": nf, "values_per_field": flen, "ms": round(ms, 4), "achieved_GBs": round(gbs, 1),
                           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    plan.transfer_metrics()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.transfer_metrics()
    out["transfer_metrics"] = {"matrix": f"{B} x {2 * info.modes}",
                               "ms": round((time.perf_counter() - t0) / reps * 1e3, 3)}
    plan.destroy()
    return out


def single_frame_bench(dh, torch, reps=10000, warm=500):
    """One 128x128 f32 frame at a time (1 pol, G=4, the smallest workload):
    the latency a caller sees for dh_process_batch of one frame followed by
    a stream synchronisation (binding call included), p50/p99 over `reps`
    calls after `warm`, and the device time of one frame's kernels."""
    cfg = dh_synth.config(0)
    f, _ = dh_synth.make_frames(cfg, n_frames=1)
    ft = torch.from_numpy(f).cuda()
    plan = dh.Plan(cfg["params"], max_batch=1)
    stream = torch.cuda.Stream()
    lat = []
    for i in range(warm + reps):
        t0 = time.perf_counter()
        plan.process(ft, 1, stream)
        stream.synchronize()
        if i >= warm:
            lat.append((time.perf_counter() - t0) * 1e3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.process(ft, 1, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plan.destroy()
    lat = np.array(lat)
    return {"workload": "1 frame 128x128 f32, 1 pol, G=4 (10 modes), process + stream sync per frame",
            "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "frames_per_s_one_at_a_time": round(1e3 / float(np.mean(lat)), 1),
            "device_ms_per_frame_back_to_back": round(e0.elapsed_time(e1) / reps, 4)}


def serving_bench(dh, torch, workers, seconds=10.0, warm=1.0, rate=5000.0, seed=220402348):
    """Serving form on the four uint16 cameras: Poisson arrivals at `rate` per
    camera from resident pools of 64 frames, continuous batching (lanes admitted
    by a 16 GiB budget, hipGraph launches). Latency = completion - arrival for
    requests arriving after the warm-up; plus the saturated rate (all requests
    at once, the second of two back-to-back runs) next to a loop that processes
    one request at a time and to static batching through the plain batch path."""
    cams = [dh_synth.config(3, c) for c in range(4)]
    pools = []
    for cfg in cams:
        f, _ = dh_synth.make_frames(cfg, n_frames=64, workers=workers)
        pools.append(torch.from_numpy(f).to("cuda:0"))
    plans = [dh.Plan(cfg["params"], max_batch=256) for cfg in cams]
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    ts, cs, ps = [], [], []
    for c in range(4):
        t = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * (seconds + warm) * 1.2)))
        t = t[t < seconds + warm]
        ts.append(t)
        cs.append(np.full(t.size, c, dtype=np.int32))
        idx = rng.integers(0, 64, size=t.size)
        base = pools[c].data_ptr()
        ps.append(base + idx.astype(np.uint64) * np.uint64(pools[c][0].nbytes))
    order = np.argsort(np.concatenate(ts), kind="stable")
    t = np.concatenate(ts)[order]
    cam = np.concatenate(cs)[order]
    ptr = np.concatenate(ps)[order]
    out = {"workload": "4 cameras uint16 (320x256 G5, 640x512 G9, 1024^2 G15, 2048^2 G20), 1 pol each, "
                       f"Poisson {rate:.0f} frames/s per camera, {warm:.0f} s warm-up + {seconds:.0f} s measured"}
    srv = dh.Server(plans, max_batch=256, hbm_budget=16 << 30, use_graphs=True)
    out["lanes"] = [srv.info(c)[0] for c in range(4)]
    done = srv.replay(t, cam, ptr)
    b, f = srv.stats()
    lat = (done - t) * 1e3
    m = t >= warm
    out["frames_per_s"] = round(float(m.sum() / (done[m].max() - warm)), 1)
    out["p50_ms"] = round(float(np.percentile(lat[m], 50)), 4)
    out["p99_ms"] = round(float(np.percentile(lat[m], 99)), 4)
    out["per_camera"] = {str(c): {"p50_ms": round(float(np.percentile(lat[m & (cam == c)], 50)), 4),
                                  "p99_ms": round(float(np.percentile(lat[m & (cam == c)], 99)), 4),
                                  "frames": int((m & (cam == c)).sum())} for c in range(4)}
    out["mean_batch"] = round(f / max(b, 1), 2)
    # saturation: every request of a 20000-request trace present at once. The
    # first such run after the light Poisson load is 10-20 % slower (lane
    # workspaces first filled at full batch size, engine clock ramping), so
    # one untimed run comes first, here and for the plain batch path below
    n = 20000
    tz = np.zeros(n)
    srv.replay(tz, cam[:n], ptr[:n])
    done = srv.replay(tz, cam[:n], ptr[:n])
    out["saturated_frames_per_s"] = round(n / float(done.max()), 1)
    srv.destroy()
    # the same 20000 requests one at a time through dh_process_batch (batch 1, waiting for each)
    t0 = time.perf_counter()
    for k in range(n):
        c = int(cam[k])
        plans[c].process(int(ptr[k]), 1, None)
        plans[c].coefs(True)
    out["one_at_a_time_frames_per_s"] = round(n / (time.perf_counter() - t0), 1)
    # the plain batch path on the same trace (static batching), and saturated
    m = t >= warm
    done_b, nb_rounds = static_batching(dh, torch, plans, pools, t, cam, max_batch=256)
    lat_b = (done_b - t) * 1e3
    out["static_batching"] = {
        "what": "the same Poisson trace through per-camera dh_process_batch: whenever the device is idle, every "
                "request that has arrived (<= 256 per camera) forms one batch per camera, the batches run on one "
                "stream and the loop waits for their coefficients; later arrivals wait for the next round. Frames "
                "are read as contiguous runs of each camera's resident pool (no gather), the plain path's best case",
        "frames_per_s": round(float(m.sum() / (done_b[m].max() - warm)), 1),
        "p50_ms": round(float(np.percentile(lat_b[m], 50)), 4), "p99_ms": round(float(np.percentile(lat_b[m], 99)), 4),
        "rounds": nb_rounds}
    static_batching(dh, torch, plans, pools, np.zeros(n), cam[:n], max_batch=256)
    done_b, nb_rounds = static_batching(dh, torch, plans, pools, np.zeros(n), cam[:n], max_batch=256)
    out["static_batching"]["saturated_frames_per_s"] = round(n / float(done_b.max()), 1)
    for p in plans:
        p.destroy()
    return out


def static_batching(dh, torch, plans, pools, t, cam, max_batch=256):
    """Replay a request trace through the plain batch path in real time: a loop
    that, whenever its previous round has finished, takes every request that
    has arrived (up to max_batch per camera), runs one dh_process_batch per
    camera on one stream and reads the coefficients back, then stamps the
    round's completion time on its requests. Returns (completion times, rounds)."""
    from collections import deque
    stream = torch.cuda.Stream()
    tiled = []
    for pool in pools:                      # contiguous runs of up to max_batch frames
        reps = -(-max_batch // pool.shape[0])
        tiled.append(pool.repeat(reps, *([1] * (pool.dim() - 1)))[:max_batch].contiguous())
    torch.cuda.synchronize()
    n = t.size
    done = np.zeros(n)
    pending = [deque() for _ in plans]
    nxt, finished, rounds = 0, 0, 0
    start = time.perf_counter()
    while finished < n:
        now = time.perf_counter() - start
        while nxt < n and t[nxt] <= now:
            pending[int(cam[nxt])].append(nxt)
            nxt += 1
        if not any(pending):
            continue
        took = []
        for c, q in enumerate(pending):
            k = min(len(q), max_batch)
            if k:
                ids = [q.popleft() for _ in range(k)]
                plans[c].process(tiled[c], k, stream)
                took.append((c, ids))
        for c, ids in took:
            plans[c].coefs(True)             # waits for the stream
        end = time.perf_counter() - start
        for c, ids in took:
            done[ids] = end
            finished += len(ids)
        rounds += 1
    return done, rounds


def camera_batches(dh, torch, workers, batch=256, steps=40, warmup=10, settle_s=0.1):
    """Batch throughput of each serving camera's plan on its own (uint16
    frames, 1 pol), with the fraction of the binding ceiling."""
    out = {}
    for c in range(4):
        cfg = dh_synth.config(3, c)
        b = batch if c < 3 else 64
        pool, _ = dh_synth.make_frames(cfg, n_frames=64, workers=workers)
        ft = torch.from_numpy(dh_synth.tile_pool(pool, b)).to("cuda:0")
        plan = dh.Plan(cfg["params"], max_batch=b)
        stream = torch.cuda.Stream()
        warm(plan, ft, b, stream, warmup, settle_s)    # a step here is 0.04-0.7 ms
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.process(ft, b, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        fps = steps * b / (e0.elapsed_time(e1) / 1e3)
        p = cfg["params"]
        out[f"{p['frame_w']}x{p['frame_h']}"] = config_fraction(
            "c4", p, plan.info, fps, f"{b} frames {p['frame_w']}x{p['frame_h']} uint16, 1 pol, G={p['max_mg']}")
        plan.destroy()
        del ft
    return out


def alignment_bench(dh, torch, workers, align_frames=50, decomp_frames=5000):
    """Alignment workload: align 50 frames 1024x1024 (2 pols, G=30) from the
    nominal tilt/defocus/waist/beam centre, then decompose 5000 frames (a pool of 250
    distinct frames tiled x20) at the aligned parameters."""
    cfg = dh_synth.config(4)
    truth = cfg["truth"]
    pool, _ = dh_synth.make_frames(cfg, n_frames=250, workers=workers)
    dev = torch.from_numpy(pool).to("cuda:0")
    frames = dev.repeat(decomp_frames // 250, 1, 1)
    plan = dh.Plan(cfg["params"], max_batch=decomp_frames)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    what = dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST | dh.ALIGN_CENTRE
    goal = plan.autoalign(frames, align_frames, dh.ALIGN_FULL, what, 1e-5)
    wall = time.perf_counter() - t0
    rep = plan.align_report()
    got = plan.params()
    bins = [1565e-9 / (512 * 20e-6) * 180 / np.pi, 1565e-9 / (1024 * 20e-6) * 180 / np.pi]
    out = {"workload": "align 50 frames 1024x1024 f32, 2 pols, G=30 from nominal (tilt, defocus, waist, "
                       "beam centre); decompose 5000 frames",
           "align_wall_s": round(wall, 4), "goal_db": round(goal, 6), "trials": rep.evaluations,
           "sweeps": rep.sweeps,
           "tilt_err_bins": [[round((got["tilt_deg"][q][a] - truth["tilt_deg"][q][a]) / bins[a], 4)
                              for a in range(2)] for q in range(2)],
           "defocus_err_D": [round(got["defocus"][q] - truth["defocus"][q], 5) for q in range(2)],
           "centre_err_px": [[round((got["beam_centre"][q][a] - truth["beam_centre"][q][a]) / 20e-6, 4)
                              for a in range(2)] for q in range(2)],
           "waist_err_pct": round(100 * (got["waist"] / truth["waist"] - 1), 3)}
    # the same alignment with the insertion loss of the batch transfer matrix
    # as the goal (each pol's tilt and defocus its own coordinate)
    plan_il = dh.Plan(cfg["params"], max_batch=align_frames)
    plan_il.set_align_goal("IL")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    il = plan_il.autoalign(frames, align_frames, dh.ALIGN_FULL, what, 1e-5)
    wall = time.perf_counter() - t0
    rep = plan_il.align_report()
    got = plan_il.params()
    plan_il.destroy()
    out["il_goal"] = {"align_wall_s": round(wall, 4), "il_db": round(il, 6), "trials": rep.evaluations,
                      "sweeps": rep.sweeps, "mdl_db": round(rep.metrics[1], 4),
                      "tilt_err_bins": [[round((got["tilt_deg"][q][a] - truth["tilt_deg"][q][a]) / bins[a], 4)
                                         for a in range(2)] for q in range(2)],
                      "defocus_err_D": [round(got["defocus"][q] - truth["defocus"][q], 5) for q in range(2)],
                      "waist_err_pct": round(100 * (got["waist"] / truth["waist"] - 1), 3)}
    # the same alignment from a zero tilt: the snap finds the off-axis term in
    # the whole Fourier plane
    plan_z = dh.Plan(dict(cfg["params"], tilt_deg=[[0.0, 0.0], [0.0, 0.0]]), max_batch=align_frames)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gz = plan_z.autoalign(frames, align_frames, dh.ALIGN_FULL, what, 1e-5)
    wall = time.perf_counter() - t0
    rep = plan_z.align_report()
    got = plan_z.params()
    plan_z.destroy()
    out["zero_tilt_start"] = {"align_wall_s": round(wall, 4), "goal_db": round(gz, 6), "trials": rep.evaluations,
                              "plane_snap_err_bins": [[round((rep.plane_tilt_deg[q][a] - truth["tilt_deg"][q][a])
                                                             / bins[a], 3) for a in range(2)] for q in range(2)],
                              "tilt_err_bins": [[round((got["tilt_deg"][q][a] - truth["tilt_deg"][q][a]) / bins[a], 4)
                                                 for a in range(2)] for q in range(2)],
                              "defocus_err_D": [round(got["defocus"][q] - truth["defocus"][q], 5) for q in range(2)],
                              "waist_err_pct": round(100 * (got["waist"] / truth["waist"] - 1), 3)}
    stream = torch.cuda.Stream()
    for _ in range(2):
        plan.process(frames, decomp_frames, stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        plan.process(frames, decomp_frames, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    out["decompose_frames_per_s"] = round(5 * decomp_frames / (e0.elapsed_time(e1) / 1e3), 1)
    out["_c5"] = config_fraction("c5", cfg["params"], plan.info, out["decompose_frames_per_s"],
                                 "5000 frames 1024x1024 f32, 2 pols, G=30 (465 modes/pol), FP32")
    plan.destroy()
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _blas():
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{t.get('internal_api')} {t.get('version')}" for t in threadpool_info() if t.get("user_api") == "blas"]
        return ", ".join(libs) or "unknown"
    except Exception:
        return "unknown"


def cpu_baseline(cfg, frames, seconds):
    """The FP64 oracle, as it stands, on a bounded sample of the same frames:
    one leg with one BLAS thread and one with every core the process may use.
    The headline object is the all-cores leg."""
    import oracle
    from threadpoolctl import threadpool_limits
    p = cfg["params"]
    g = oracle.geometry(p)
    ncores = len(os.sched_getaffinity(0))
    legs = []
    for threads in (1, ncores):
        with threadpool_limits(limits=threads):
            oracle.process_frame(frames[0].astype(np.float64), p, g)   # warm caches
            n = 0
            t0 = time.perf_counter()
            while n < frames.shape[0] and (n < 2 or time.perf_counter() - t0 < seconds):
                oracle.process_frame(frames[n].astype(np.float64), p, g)
                n += 1
            dt = time.perf_counter() - t0
        legs.append({"value": n / dt, "unit": "frames/s", "cores": threads, "frames": n, "seconds": round(dt, 2)})
    cpu, blas = _cpu_model(), _blas()
    all_cores = legs[1]
    return {"value": all_cores["value"], "unit": "frames/s", "cores": all_cores["cores"], "kind": "oracle",
            "sample": f"{all_cores['frames']} frames of the same batch, one at a time, {all_cores['seconds']} s "
                      f"({ncores} BLAS threads); single-thread leg {legs[0]['frames']} frames in {legs[0]['seconds']} s",
            "cpu_model": cpu, "blas": blas, "legs": legs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # defaults: 50 warm-up steps (~35 ms) reach the steady engine clock, which
    # the VALU-bound column pass needs (its time drops ~25 % over the first
    # ~20 ms of sustained work); 100 timed steps (~65 ms)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--settle-ms", type=float, default=150.0,
                    help="untimed steps for this long before the warm-up steps (engine clock ramp)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 / split BF16 / split FP16 comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the four-camera serving run")
    ap.add_argument("--no-align", action="store_true", help="skip the alignment workload")
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
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(frames would shard by frame with no exchange).", file=sys.stderr)
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
    # the engine clock ramps up over the first ~20 ms of sustained work (the
    # VALU-bound column pass runs ~25 % slower before): untimed steps until
    # --settle-ms of device work have passed, then the W warm-up steps
    settle = 0
    t_settle = time.perf_counter()
    while (time.perf_counter() - t_settle) * 1e3 < args.settle_ms:
        plan.process(ft, B, stream)
        stream.synchronize()
        settle += 1
    for _ in range(args.warmup):
        plan.process(ft, B, stream)
    stream.synchronize()
    print(f"[bench] clock settle {settle} steps, warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # timed window 1: the throughput (one event pair per step, for the latency)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        starts[k].record(stream)
        plan.process(ft, B, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    total_ms = starts[0].elapsed_time(ends[-1])
    value = args.steps * B / (total_ms / 1e3)
    print(f"[bench] timed {args.steps} steps: {total_ms:.2f} ms", file=sys.stderr, flush=True)
    # timed window 2, right after, same K steps: HIP events around every launch
    # on the stream it runs on (the stage breakdown and the roofline). The
    # extra event records add ~3 % to a step, so they stay out of window 1.
    plan.set_stage_timing(True)
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0.record(stream)
    for k in range(args.steps):
        plan.process(ft, B, stream)
    w1.record(stream)
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.set_stage_timing(False)
    stage_window_ms = w0.elapsed_time(w1) / args.steps

    # roofline of the dominant kernel: the path's algorithmic bytes (each frame
    # read once, its coefficients written once) for the frames one launch
    # processes, over the kernel's mean launch time
    sb = stage_bytes(info, cfg["params"], B)
    dom = max(stages, key=lambda k: stages[k][0])
    ms_dom, n_dom = stages[dom]
    frames_per_launch = B / (n_dom / args.steps)
    alg_frame = algorithmic_bytes_per_frame(cfg["params"], info)
    per_launch_bytes = alg_frame * frames_per_launch
    launch_s = ms_dom / n_dom / 1e3
    achieved = per_launch_bytes / launch_s / 1e9
    traffic = counter_traffic(dom, info, frames_per_launch) if B == 1000 else None
    kernel_bytes = sb[dom] / (n_dom / args.steps)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes": round(per_launch_bytes),
                "algorithmic_bytes_per_frame": int(alg_frame),
                "algorithmic_what": "frame read once + raw coefficients written once, per frame of the launch",
                "kernel": dom, "launch_ms": round(ms_dom / n_dom, 4), "launches_per_step": n_dom // args.steps,
                "kernel_bytes": round(kernel_bytes),
                "kernel_bytes_what": "what the kernel reads and writes by design (frame in, row-pass spectrum out)",
                "kernel_bytes_frac": round(kernel_bytes / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_over_algorithmic": round(traffic / per_launch_bytes, 3) if traffic else None}
    step_s = total_ms / args.steps / 1e3
    fft_ms = (stages["row_fft"][0] + stages["column_fft_window"][0]) / args.steps
    path = {"what": "whole path: frames x algorithmic bytes per frame over the timed step",
            "achieved_GBs": round(B * alg_frame / step_s / 1e9, 1),
            "frac": round(B * alg_frame / step_s / 1e9 / HBM_PEAK_GBS, 4),
            "ceiling_frames_per_s": round(HBM_PEAK_GBS * 1e9 / alg_frame, 1),
            "fft_stages_frac": round(B * frame_bytes_of(cfg["params"]) / (fft_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "fft_stages_what": "frame bytes over the row + column pass time (stage window)"}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1000 frames 640x512 f32, 2 pols (320x512 windows), G=9 (45 modes/pol), "
                               "defocus, shot+read noise; plain FP32",
                   "frames": B, "frame": "640x512", "pols": 2, "max_mg": 9, "precision": "fp32",
                   "path": {1: "field", 2: "spectral"}[info.path]},
        "clock_settle_steps": settle,
        "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "stage_window": {"what": "a second timed window of the same K steps right after the first, with HIP "
                                 "events around every launch; stages_ms_per_step and roofline come from it",
                         "ms_per_step": round(stage_window_ms, 4)},
        "path_roofline": path,
        "roofline": roofline,
        "configs_roofline": {"c2": config_fraction("c2", cfg["params"], info, value, "1000 frames 640x512 f32, "
                                                   "2 pols, G=9 (45 modes/pol), FP32 (this line's value)")},
    }
    plan.destroy()
    if not args.no_forms:
        out["forms"] = time_forms(dh, torch, cfg, ft, B, stream)
        out["variants"] = time_variants(dh, torch, cfg, ft, B, stream)
        out["aux"] = time_aux(dh, torch, cfg, ft, B, stream)
        out["configs_roofline"]["c3"] = out["forms"].pop("_c3", None)
        print("[bench] forms done", file=sys.stderr, flush=True)
    del ft
    if not args.no_serving:
        out["single_frame"] = single_frame_bench(dh, torch)
        out["serving"] = serving_bench(dh, torch, workers)
        out["configs_roofline"]["c4"] = camera_batches(dh, torch, workers)
        print("[bench] serving done", file=sys.stderr, flush=True)
    if not args.no_align:
        out["alignment"] = alignment_bench(dh, torch, workers)
        out["configs_roofline"]["c5"] = out["alignment"].pop("_c5", None)
        print("[bench] alignment done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, frames, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
