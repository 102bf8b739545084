"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Tolerance (FP32 path): relative L2 error <= 1e-5 per frame and polarisation
on the Fourier window, the field and the coefficients (raw and normalised).
"""
import math
import os
import sys

import numpy as np
import pytest

import dh_synth
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)


def run_gpu(params, frames, keep=True, chunk=None, stream=True, path="auto"):
    """Process `frames` through the C ABI. keep: also return the Fourier
    window and (where the path forms it) the field."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    fields = keep and path != "spectral"
    d = dict(params, keep_window=int(keep), keep_fields=int(fields), path=path)
    if chunk:
        os.environ["DH_CHUNK_FRAMES"] = str(chunk)
    try:
        plan = dh.Plan(d, max_batch=frames.shape[0])
    finally:
        os.environ.pop("DH_CHUNK_FRAMES", None)
    ft = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    s = torch.cuda.Stream() if stream else None
    if s is not None:
        s.wait_stream(torch.cuda.current_stream())
    plan.process(ft, frames.shape[0], s)
    out = dict(coefs=plan.coefs(False), coefs_norm=plan.coefs(True), info=plan.info)
    if keep:
        out["window"] = plan.window()
    if fields:
        out["field"] = plan.fields()
    torch.cuda.synchronize()
    plan.destroy()
    return out


def check_frames(params, frames, gpu, idx, keep=True, tol=TOL):
    worst = {}
    for i in idx:
        ref = oracle.process_frame(frames[i].astype(np.float64), params)
        keys = ["coefs", "coefs_norm"] + [k for k in ("window", "field") if keep and k in gpu]
        for k in keys:
            for pol in range(params["pol_count"]):
                if params["max_mg"] == 0 and k.startswith("coefs"):
                    continue
                e = _rel(gpu[k][i][pol].astype(np.complex128), ref[k][pol])
                worst[k] = max(worst.get(k, 0.0), e)
    _say("worst rel-L2", {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (k, v)
    return worst


def _frames(idx, cam=0, n=None, first=0):
    cfg = dh_synth.config(idx, cam)
    f, c = dh_synth.make_frames(cfg, n_frames=n, first=first)
    return cfg, f, c


def test_config0_single_frame():
    cfg, f, _ = _frames(0)
    _say("config0 128x128 G=4 batch 1")
    gpu = run_gpu(cfg["params"], f)
    check_frames(cfg["params"], f, gpu, [0])


def test_config1_small_batch_ragged_chunks():
    cfg, f, _ = _frames(1, n=7)
    _say("config1 640x512 2 pols G=9 batch 7 chunk 3")
    gpu = run_gpu(cfg["params"], f, chunk=3)
    check_frames(cfg["params"], f, gpu, range(7))


def test_config1_full_batch_sampled():
    cfg, pool, _ = _frames(1, n=100)
    f = dh_synth.tile_pool(pool, 1000)
    _say("config1 batch 1000 (bench launch configuration), sampled frames")
    gpu = run_gpu(cfg["params"], f, keep=False)
    check_frames(cfg["params"], f, gpu, [0, 1, 85, 86, 511, 998, 999], keep=False)


def test_config2_g20():
    cfg, f, _ = _frames(2)
    _say("config2 128x128 G=20")
    gpu = run_gpu(cfg["params"], f)
    check_frames(cfg["params"], f, gpu, [0])


@pytest.mark.parametrize("cam", [0, 1, 2, 3])
def test_config3_cameras_u16(cam):
    cfg, f, _ = _frames(3, cam=cam, n=3 if cam < 3 else 2)
    assert f.dtype == np.uint16
    _say("config3 camera", cam, f.shape)
    gpu = run_gpu(cfg["params"], f)
    check_frames(cfg["params"], f, gpu, range(f.shape[0]))


def test_config4_alignment_shape():
    cfg, f, _ = _frames(4, n=3)
    _say("config4 1024x1024 2 pols G=30 at the true parameters")
    gpu = run_gpu(cfg["truth"], f)
    check_frames(cfg["truth"], f, gpu, range(3))


def run_gpu_tiled(params, pool, n):
    """Process n frames (frame i = pool[i % len(pool)], tiled on the device)
    in one dh_process_batch call with max_batch = n, as the benchmark launches
    them (the library's own launch chunks); returns the coefficients."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    plan = dh.Plan(dict(params, keep_window=0, keep_fields=0), max_batch=n)
    dev = torch.from_numpy(np.ascontiguousarray(pool)).cuda()
    ft = dev.repeat(-(-n // pool.shape[0]), *([1] * (dev.dim() - 1)))[:n].contiguous()
    del dev
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.process(ft, n, s)
    out = dict(coefs=plan.coefs(False), coefs_norm=plan.coefs(True), chunk=plan.info.chunk)
    torch.cuda.synchronize()
    plan.destroy()
    del ft
    return out


def check_tiled(params, pool, gpu, idx, tol=TOL):
    """Sampled frames of a tiled batch against the oracle (each distinct pool
    frame computed once)."""
    worst, refs = {}, {}
    for i in idx:
        q = i % pool.shape[0]
        if q not in refs:
            refs[q] = oracle.process_frame(pool[q].astype(np.float64), params)
        for k in ("coefs", "coefs_norm"):
            for pol in range(params["pol_count"]):
                worst[k] = max(worst.get(k, 0.0), _rel(gpu[k][i][pol].astype(np.complex128), refs[q][k][pol]))
    _say("worst rel-L2", {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (k, v)


def test_config2_g20_full_batch_sampled():
    """The G = 20 throughput form at the 640x512 batch shape: 1000 frames in
    one call, as timed by the benchmark."""
    cfg, pool, _ = _frames(1, n=10)
    params = dict(cfg["params"], max_mg=20)
    _say("640x512 2 pols G=20 batch 1000 (benchmark launch), sampled frames")
    gpu = run_gpu_tiled(params, pool, 1000)
    check_tiled(params, pool, gpu, [0, 1, 499, 500, 998, 999])


@pytest.mark.parametrize("cam", [0, 1, 2, 3])
def test_config3_cameras_full_batch_sampled(cam):
    """Each camera's batch as the benchmark times it (256 frames, 64 for the
    2048 x 2048 camera), uint16 pixels."""
    cfg, pool, _ = _frames(3, cam=cam, n=4 if cam < 3 else 2)
    n = 256 if cam < 3 else 64
    _say("camera", cam, "batch", n, "(benchmark launch), sampled frames")
    gpu = run_gpu_tiled(cfg["params"], pool, n)
    check_tiled(cfg["params"], pool, gpu, [0, 1, n // 2 + 1, n - 1])


def test_config4_decomposition_full_batch_sampled():
    """The 5000-frame 1024x1024 two-pol G = 30 decomposition in one call: the
    library splits it into launch chunks (2 GiB of workspace each); frames on
    both sides of every chunk boundary against the oracle."""
    cfg, pool, _ = _frames(4, n=3)
    n = 5000
    _say("1024x1024 2 pols G=30 batch 5000 (benchmark launch), frames at the chunk boundaries")
    gpu = run_gpu_tiled(cfg["truth"], pool, n)
    c = gpu["chunk"]
    assert 0 < c < n, c
    idx = sorted({0, n - 1} | {i for k in range(c, n, c) for i in (k - 1, k)})
    check_tiled(cfg["truth"], pool, gpu, idx)


def test_subpixel_centre_defocus_and_per_pol_tilt():
    cfg = dh_synth.config(1)
    # 256x256 windows inside the 320x512 halves, so the beam centres can move
    truth = dict(cfg["truth"], fft_w=256, fft_h=256, defocus=[0.15, -0.1],
                 tilt_deg=[[1.45, 1.55], [1.52, 1.47]],
                 beam_centre=[[0.3 * 20e-6, -2.2 * 20e-6], [-1.4 * 20e-6, 0.1 * 20e-6]])
    cfg = dict(cfg, truth=truth)
    f, c = dh_synth.make_frames(cfg, n_frames=2)
    _say("sub-pixel centre / defocus / per-pol tilt")
    gpu = run_gpu(truth, f)
    check_frames(truth, f, gpu, range(2))


def test_no_decomposition_fields_only():
    cfg, f, _ = _frames(0)
    p = dict(cfg["params"], max_mg=0)
    _say("G=0 fields only")
    gpu = run_gpu(p, f)
    assert gpu["coefs"].shape[2] == 0
    check_frames(p, f, gpu, [0])


def test_frame_alone_equals_frame_in_batch():
    cfg, f, _ = _frames(1, n=6)
    _say("determinism: alone vs in batch")
    alone = run_gpu(cfg["params"], f[3:4], keep=False)
    batch = run_gpu(cfg["params"], f, keep=False, chunk=4)
    assert np.array_equal(alone["coefs"][0], batch["coefs"][3])
    assert np.array_equal(alone["coefs_norm"][0], batch["coefs_norm"][3])


def _small_cfg(kind):
    """128x128 transforms: recipe 0 (G=4), recipe 2 (G=20, two mode tiles),
    a 256x128 frame with two pols (G=9), and recipe 0 as uint16 (G=6)."""
    from dh_synth.holograms import _base_params
    if kind == "g4":
        return dh_synth.config(0)
    if kind == "g20":
        return dh_synth.config(2)
    cfg = dict(dh_synth.config(0))
    if kind == "2pol":
        p = _base_params(256, 128, 2, 128, 128, 200e-6, 9)
    else:
        p = _base_params(128, 128, 1, 128, 128, 200e-6, 6, dtype="u16")
    cfg.update(params=p, truth=dict(p), dtype=p["input_dtype"])
    return cfg


@pytest.mark.parametrize("kind", ["g4", "g20", "2pol", "u16"])
def test_small_frames_alone_equal_in_batch(kind):
    """128-point transforms (one pol, two pols, one and two mode tiles, f32
    and uint16): every frame of a 20-frame batch equals the same frame
    processed alone, bit for bit (window too), and the frames match the
    oracle."""
    cfg = _small_cfg(kind)
    f, _ = dh_synth.make_frames(cfg, n_frames=20)
    p = cfg["params"]
    _say(f"small frames {kind}: batch of 20 vs alone")
    big = run_gpu(p, f, keep=True, path="spectral")
    for i in (0, 7, 19):
        alone = run_gpu(p, f[i:i + 1], keep=True, path="spectral")
        assert np.array_equal(big["coefs"][i], alone["coefs"][0]), i
        assert np.array_equal(big["coefs_norm"][i], alone["coefs_norm"][0]), i
        assert np.array_equal(big["window"][i], alone["window"][0]), i
    check_frames(p, f, big, [0, 19])


@pytest.mark.parametrize("path", ["field", "spectral"])
@pytest.mark.parametrize("idx", [0, 1])
def test_largest_group_count(idx, path):
    """G = 32, the most the plan takes (528 modes per pol), on both paths."""
    cfg, f, _ = _frames(idx, n=2 if idx else 1)
    p = dict(cfg["params"], max_mg=32)
    _say("G=32 recipe %d, %s path" % (idx, path))
    gpu = run_gpu(p, f, keep=path == "field", path=path)
    assert gpu["coefs"].shape[2] == 528
    check_frames(p, f, gpu, range(f.shape[0]), keep=path == "field")


@pytest.mark.parametrize("idx,cam,g,n", [
    (1, 0, 33, 2),       # 640x512, 2 pols: 64 mode columns, the second chunk mostly padding
    (1, 0, 64, 2),       # two full chunks
    (0, 0, 48, 1),       # 128x128: 16 box columns per workgroup, two A-row tiles
    (3, 2, 40, 1),       # 1024x1024 u16 camera: 1024-point columns with mode chunks (4 per workgroup)
    (4, 0, 30, 1),       # 1024x1024, 2 pols, G=30: 1024-point columns, 8 per workgroup, two mode tiles
    (3, 3, 64, 1),       # 2048x2048 u16 camera, W = 672
    (3, 3, 100, 1),      # the largest group count: 5050 modes per pol, four chunks
])
def test_large_group_counts(idx, cam, g, n):
    """G above 32 on the spectral path (mode columns contracted in chunks of
    32 over the window held in LDS): coefficients and window against the
    oracle."""
    cfg, f, _ = _frames(idx, cam, n=n)
    p = dict(cfg["params"], max_mg=g)
    _say(f"G={g} recipe {idx} camera {cam}, {n} frames, spectral path")
    gpu = run_gpu(p, f, keep=True, path="spectral")
    assert gpu["coefs"].shape[2] == g * (g + 1) // 2
    check_frames(p, f, gpu, range(n))


def test_lg_basis_at_100_groups():
    """The LG basis at the paper's largest group count on the 2048x2048
    camera: coefficients (raw and normalised) against the oracle's HG
    coefficients times its per-group HG->LG blocks."""
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(3, 3, n=1)
    p = dict(cfg["params"], max_mg=100)
    _say("LG basis, G=100, 2048x2048 camera")
    raw, nrm, _ = _basis_run(p, f, dh.BASIS_LG)
    assert raw.shape == (1, 1, 5050)
    blocks = oracle.lg_blocks(100)
    ref = oracle.process_frame(f[0].astype(np.float64), p)
    lr, ln = oracle.apply_lg_blocks(ref["coefs"], blocks), oracle.apply_lg_blocks(ref["coefs_norm"], blocks)
    e, en = _rel(raw[0][0].astype(np.complex128), lr[0]), _rel(nrm[0][0].astype(np.complex128), ln[0])
    _say(f"LG rel-L2 raw {e:.2e}, normalised {en:.2e}")
    assert e <= TOL and en <= TOL


def test_mode0_large_group_count():
    """IFFT mode 0 with G = 64 (coefficients from the spectral tables on the
    FFT grid, fields exported) against the oracle."""
    cfg, f, _ = _frames(1, n=2)
    p = dict(cfg["params"], max_mg=64, ifft_mode=0)
    _say("mode 0, G=64, 640x512")
    gpu = run_gpu(p, f, keep=False, path="spectral")
    check_frames(p, f, gpu, range(2), keep=False)


def test_zero_frames_give_zero_not_nan():
    """All-zero frames: every coefficient, raw and normalised (power 0), is
    exactly zero on both paths, and the int16 export has scale 1."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(1)
    f = np.zeros((3, 512, 640), dtype=np.float32)
    ft = torch.from_numpy(f).cuda()
    for path in ("field", "spectral"):
        _say("zero frames, %s path" % path)
        plan = dh.Plan(dict(cfg["params"], path=path, keep_fields=int(path == "field")), max_batch=3)
        plan.process(ft, 3, None)
        for normalised in (False, True):
            c = plan.coefs(normalised)
            assert np.all(c == 0) and not np.any(np.isnan(c))
        if path == "field":
            re, im, sc = plan.fields16()
            assert not re.any() and not im.any() and np.all(sc == 1.0)
        plan.destroy()


# ---------------------------------------------------------------- spectral path
@pytest.mark.parametrize("idx,cam,n,chunk", [
    (0, 0, 1, None),      # 128x128 G=4
    (1, 0, 7, 3),         # 640x512 2 pols G=9, ragged chunks
    (2, 0, 1, None),      # 128x128 G=20: two n-tiles
    (3, 0, 3, None),      # 320x256 uint16 G=5
    (3, 1, 3, None),      # 640x512 uint16 G=9
    (3, 2, 2, None),      # 1024x1024 uint16 G=15
    (3, 3, 1, None),      # 2048x2048 uint16 G=20
    (4, 0, 2, None),      # 1024x1024 2 pols G=30
])
def test_spectral_path_vs_oracle(idx, cam, n, chunk):
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(idx, cam=cam, n=n)
    _say("spectral path recipe", idx, "camera", cam, f.shape)
    gpu = run_gpu(cfg["params"], f, chunk=chunk, path="spectral")
    assert gpu["info"].path == dh.PATH_SPECTRAL
    check_frames(cfg["params"], f, gpu, range(n))


def test_spectral_path_subpixel_centre_defocus_per_pol_tilt():
    cfg = dh_synth.config(1)
    truth = dict(cfg["truth"], fft_w=256, fft_h=256, defocus=[0.15, -0.1],
                 tilt_deg=[[1.45, 1.55], [1.52, 1.47]],
                 beam_centre=[[0.3 * 20e-6, -2.2 * 20e-6], [-1.4 * 20e-6, 0.1 * 20e-6]])
    f, _ = dh_synth.make_frames(dict(cfg, truth=truth), n_frames=2)
    _say("spectral path: sub-pixel centre / defocus / per-pol tilt")
    gpu = run_gpu(truth, f, path="spectral")
    check_frames(truth, f, gpu, range(2))


def test_field_and_spectral_paths_agree():
    cfg, pool, _ = _frames(1, n=50)
    f = dh_synth.tile_pool(pool, 300)
    _say("field vs spectral path, 640x512 batch 300")
    a = run_gpu(cfg["params"], f, keep=False, path="field")
    b = run_gpu(cfg["params"], f, keep=False, path="spectral")
    worst = max(_rel(b["coefs"][i][q].astype(np.complex128), a["coefs"][i][q].astype(np.complex128))
                for i in range(f.shape[0]) for q in range(2))
    _say("worst rel-L2 between the paths %.2e" % worst)
    assert worst <= 2 * TOL


@pytest.mark.parametrize("path", ["spectral", "field"])
def test_row_pass_ragged_tile_count(path):
    """128x64 frames: the row pass's one 64-row tile per frame and pol, with two
    tiles per workgroup on a grid this large, so every workgroup's second tile
    is past the last row (loads clamped, nothing stored). Each frame equals the
    same frame processed alone (one tile per workgroup), bit for bit, and the
    oracle."""
    cfg = dh_synth.config(0)
    p = dict(cfg["params"], frame_h=64, fft_h=64)
    pool, _ = dh_synth.make_frames(dict(cfg, params=p, truth=p), n_frames=8)
    f = dh_synth.tile_pool(pool, 4100)
    _say("ragged tile count: 4100 frames 128x64,", path)
    big = run_gpu(dict(p, path=path), f, keep=False, path=path)
    for i in range(8):
        alone = run_gpu(dict(p, path=path), f[i:i + 1], keep=False, path=path)
        for k in (i, i + 8 * 256, i + 8 * 511):
            assert np.array_equal(big["coefs"][k], alone["coefs"][0]), (i, k)
    check_frames(p, f, big, [0, 4099], keep=False)


# ---------------------------------------------------------------- precision form
TOL_SPLIT = 1e-4


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("idx,n,groups", [(2, 1, 20), (0, 1, 4), (1, 3, 9), (1, 3, 20), (4, 2, 30)])
def test_precision_forms(prec, idx, n, groups):
    cfg = dh_synth.config(idx)
    p = dict(cfg["truth"], max_mg=groups, precision=prec)
    f, _ = dh_synth.make_frames(cfg, n_frames=n)
    _say("precision form", prec, "recipe", idx, "G", groups)
    gpu = run_gpu(p, f)
    check_frames(p, f, gpu, range(n), tol=TOL_SPLIT)


def test_precision_report_per_result():
    """Per-frame coefficient error of each form vs the FP64 oracle at the
    G=20 shapes (128x128 and 640x512): max and p99 over the frames."""
    rows = []
    for idx, n in [(2, 1), (1, 8)]:
        cfg = dh_synth.config(idx)
        f, _ = dh_synth.make_frames(cfg, n_frames=n)
        base = dict(cfg["truth"], max_mg=20)
        refs = [oracle.process_frame(f[i].astype(np.float64), base)["coefs_norm"] for i in range(n)]
        for prec in ["fp32", "split_bf16", "split_fp16"]:
            gpu = run_gpu(dict(base, precision=prec), f, keep=False)
            errs = np.array([_rel(gpu["coefs_norm"][i].astype(np.complex128), refs[i]) for i in range(n)])
            rows.append((idx, prec, float(errs.max()), float(np.percentile(errs, 99))))
    for r in rows:
        _say("precision report recipe %d %-10s max %.2e p99 %.2e" % r)
    for idx, prec, mx, _ in rows:
        assert mx <= (TOL if prec == "fp32" else TOL_SPLIT), (idx, prec, mx)


# ---------------------------------------------------------------- alignment
def _align_plan(params, f):
    torch = _torch()
    import paper_2204_02348_amd as dh
    plan = dh.Plan(params, max_batch=f.shape[0])
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    return dh, plan, ft


def test_alignment_goal_matches_oracle():
    cfg = dh_synth.config(4)
    f, _ = dh_synth.make_frames(cfg, n_frames=3)
    truth = cfg["truth"]
    off = dict(truth, tilt_deg=[[truth["tilt_deg"][0][0] + 0.01, truth["tilt_deg"][0][1]], truth["tilt_deg"][1]],
               defocus=[truth["defocus"][0], truth["defocus"][1] + 0.03], waist=truth["waist"] * 1.02)
    for p in (truth, off):
        _say("alignment goal parity", p["tilt_deg"], p["defocus"], p["waist"])
        dh, plan, ft = _align_plan(p, f)
        g = plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_TWEAK, what=0)
        ref = oracle.goal_db(f, p)
        plan.destroy()
        _say("goal gpu %.7f dB oracle %.7f dB" % (g, ref))
        assert abs(10 ** (g / 10) - 10 ** (ref / 10)) <= 1e-5 * 10 ** (ref / 10)


def test_alignment_snap_finds_the_tilt():
    cfg = dh_synth.config(4)
    f, _ = dh_synth.make_frames(cfg, n_frames=10)
    dh, plan, ft = _align_plan(cfg["params"], f)
    _say("alignment snap from nominal")
    plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_ESTIMATE, what=dh.ALIGN_TILT)
    got = plan.params()["tilt_deg"]
    plan.destroy()
    bins = [1565e-9 / (512 * 20e-6) / oracle.DEG, 1565e-9 / (1024 * 20e-6) / oracle.DEG]
    for q in range(2):
        for a in range(2):
            err = abs(got[q][a] - cfg["truth"]["tilt_deg"][q][a]) / bins[a]
            _say("snap pol %d axis %d error %.2f bins" % (q, a, err))
            assert err < 3.0


@pytest.mark.parametrize("idx,cam", [(1, 0), (3, 1)])
def test_alignment_plane_snap_matches_oracle(idx, cam):
    """The snap's first guess from the whole Fourier plane (ESTIMATE, tilt),
    from a zero starting tilt, against the oracle's on the same frames:
    640x512 f32 with 2 pols, and the 640x512 uint16 camera."""
    cfg, f, _ = _frames(idx, cam=cam, n=6)
    start = dict(cfg["params"], tilt_deg=[[0.0, 0.0]] * cfg["params"]["pol_count"])
    ref = oracle.snap_tilt_plane(f, start)
    dh, plan, ft = _align_plan(start, f)
    _say("plane snap, recipe", idx, "camera", cam, f.shape)
    plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_ESTIMATE, what=dh.ALIGN_TILT)
    rep = plan.align_report()
    plan.destroy()
    p = cfg["params"]
    bins = [p["wavelength"] / (p["fft_w"] * p["pixel_size"]) / oracle.DEG,
            p["wavelength"] / (p["fft_h"] * p["pixel_size"]) / oracle.DEG]
    for q in range(p["pol_count"]):
        for a in range(2):
            err = abs(rep.plane_tilt_deg[q][a] - ref[q][a]) / bins[a]
            _say("pol %d axis %d: gpu %.5f oracle %.5f deg (%.4f bins apart), truth %.5f" % (
                q, a, rep.plane_tilt_deg[q][a], ref[q][a], err, cfg["truth"]["tilt_deg"][q][a]))
            assert err < 0.01


def test_alignment_full_from_a_zero_tilt():
    """FULL alignment starting from a zero tilt (the snap finds the off-axis
    term in the whole Fourier plane) recovers the truth (1024x1024, 2 pols,
    G=30)."""
    cfg = dh_synth.config(4)
    n = 20
    f, _ = dh_synth.make_frames(cfg, n_frames=n)
    truth = cfg["truth"]
    dh, plan, ft = _align_plan(dict(cfg["params"], tilt_deg=[[0.0, 0.0], [0.0, 0.0]]), f)
    _say("alignment full from a zero tilt, %d frames" % n)
    plan.autoalign(ft, n, mode=dh.ALIGN_FULL, what=dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST, tol=1e-5)
    rep = plan.align_report()
    got = plan.params()
    plan.destroy()
    bins = [1565e-9 / (512 * 20e-6) / oracle.DEG, 1565e-9 / (1024 * 20e-6) / oracle.DEG]
    for q in range(2):
        _say("pol %d plane snap %.4f %.4f, final tilt err %.3f / %.3f bins" % (
            q, rep.plane_tilt_deg[q][0], rep.plane_tilt_deg[q][1],
            (got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) / bins[0],
            (got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) / bins[1]))
        assert abs(got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) < 0.3 * bins[0]
        assert abs(got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) < 0.3 * bins[1]
        assert abs(got["defocus"][q] - truth["defocus"][q]) < 0.01
    assert abs(got["waist"] / truth["waist"] - 1) < 0.01


def test_alignment_defocus_snap_matches_oracle():
    """ESTIMATE on the defocus alone, at the true tilt, centre and waist and a
    zero defocus: the snap's magnitude per pol against the oracle's (1024x1024,
    2 pols, G=30); the kept defocus is one of 0, +|D|, -|D|."""
    cfg = dh_synth.config(4)
    f, _ = dh_synth.make_frames(cfg, n_frames=3)
    truth = cfg["truth"]
    start = dict(truth, defocus=[0.0, 0.0])
    ref = oracle.snap_defocus_magnitude(f, start, truth["waist"])
    dh, plan, ft = _align_plan(start, f)
    plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_ESTIMATE, what=dh.ALIGN_DEFOCUS)
    rep = plan.align_report()
    got = plan.params()["defocus"]
    plan.destroy()
    for q in range(2):
        _say("pol %d |D| gpu %.6f oracle %.6f, kept %.5f, truth %.5f" % (
            q, rep.snap_defocus[q], ref[q], got[q], truth["defocus"][q]))
        assert abs(rep.snap_defocus[q] - ref[q]) <= 1e-4 * max(1.0, ref[q])
        assert min(abs(got[q]), abs(got[q] - rep.snap_defocus[q]), abs(got[q] + rep.snap_defocus[q])) < 1e-12


def test_alignment_recovers_truth_and_then_processes():
    cfg = dh_synth.config(4)
    n = 20
    f, _ = dh_synth.make_frames(cfg, n_frames=n)
    truth = cfg["truth"]
    dh, plan, ft = _align_plan(cfg["params"], f)
    _say("alignment full from nominal, %d frames" % n)
    g = plan.autoalign(ft, n, mode=dh.ALIGN_FULL, what=dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST, tol=1e-5)
    rep = plan.align_report()
    got = plan.params()
    bins = [1565e-9 / (512 * 20e-6) / oracle.DEG, 1565e-9 / (1024 * 20e-6) / oracle.DEG]
    _say("goal %.5f dB (after snap %.5f), %d trials, %d sweeps" % (g, rep.start_goal_db, rep.evaluations, rep.sweeps))
    for q in range(2):
        _say("pol %d tilt err %.3f / %.3f bins, defocus err %.4f D" % (
            q, (got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) / bins[0],
            (got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) / bins[1], got["defocus"][q] - truth["defocus"][q]))
    _say("waist err %.4f %%" % (100 * (got["waist"] / truth["waist"] - 1)))
    ref_truth = oracle.goal_db(f, truth, indices=range(4))
    _say("oracle goal at the truth (4 frames) %.5f dB" % ref_truth)
    for q in range(2):
        assert abs(got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) < 0.3 * bins[0]
        assert abs(got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) < 0.3 * bins[1]
        assert abs(got["defocus"][q] - truth["defocus"][q]) < 0.01
    assert abs(got["waist"] / truth["waist"] - 1) < 0.01
    # the aligned plan processes frames; its coefficients match the oracle at the aligned parameters
    aligned = dict(truth, tilt_deg=got["tilt_deg"], defocus=got["defocus"], waist=got["waist"])
    plan.process(ft, n, None)
    coefs = plan.coefs(False)
    plan.destroy()
    for i in (0, n - 1):
        ref = oracle.process_frame(f[i].astype(np.float64), aligned)["coefs"]
        for pol in range(2):
            assert _rel(coefs[i][pol].astype(np.complex128), ref[pol]) <= TOL



# ---------------------------------------------------------------- serving
def _cameras(n_frames):
    """The four serving cameras (uint16) with a small pool of frames each."""
    cams = []
    for cam in range(4):
        cfg = dh_synth.config(3, cam)
        f, _ = dh_synth.make_frames(cfg, n_frames=n_frames if cam < 3 else 2)
        cams.append((cfg, f))
    return cams


def _trace(n, counts, rate, seed):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    cam = rng.integers(0, 4, size=n).astype(np.int32)
    idx = np.array([rng.integers(0, counts[c]) for c in cam])
    return t, cam, idx


@pytest.mark.parametrize("graphs", [True, False])
def test_serving_result_alone_equals_in_the_mix(graphs):
    torch = _torch()
    import paper_2204_02348_amd as dh
    cams = _cameras(4)
    plans = [dh.Plan(cfg["params"], max_batch=64) for cfg, _ in cams]
    pools = [torch.from_numpy(f).cuda() for _, f in cams]
    counts = [f.shape[0] for _, f in cams]
    srv = dh.Server(plans, max_batch=64, hbm_budget=8 << 30, use_graphs=graphs)
    _say("serving graphs=%s lanes %s" % (graphs, [srv.info(c)[0] for c in range(4)]))
    n = 600
    t, cam, idx = _trace(n, counts, 40000.0, 7)
    ptrs = [pools[c][i].data_ptr() for c, i in zip(cam, idx)]
    per = [srv.info(c)[2] for c in range(4)]
    res = [np.zeros(per[c], dtype=np.complex64) for c in cam]
    torch.cuda.synchronize()          # pools uploaded before the lanes' streams read them
    done = srv.replay(t, cam, ptrs, res)
    batches, frames = srv.stats()
    _say("served %d frames in %d batches; latency p50 %.1f us p99 %.1f us" % (
        frames, batches, 1e6 * np.percentile(done - t, 50), 1e6 * np.percentile(done - t, 99)))
    assert np.all(done >= t) and frames == n
    assert batches < n      # requests were batched together
    srv.destroy()
    # every result equals the same frame processed alone, bit for bit
    alone = {}
    for c in range(4):
        for i in range(counts[c]):
            plans[c].process(pools[c][i], 1, None)
            alone[(c, i)] = plans[c].coefs(True)[0].reshape(-1)
    for k in range(n):
        assert np.array_equal(res[k], alone[(int(cam[k]), int(idx[k]))]), k
    # and matches the oracle
    for c in range(4):
        cfg, f = cams[c]
        ref = oracle.process_frame(f[0].astype(np.float64), cfg["params"])["coefs_norm"].reshape(-1)
        assert _rel(alone[(c, 0)].astype(np.complex128), ref) <= TOL
    for p in plans:
        p.destroy()


def test_serving_admission_by_budget():
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(3, 1)
    plan = dh.Plan(cfg["params"], max_batch=32)
    srv = dh.Server([plan], max_batch=32, hbm_budget=0)
    lanes, nbytes, _ = srv.info(0)
    srv.destroy()
    assert lanes == 4
    srv = dh.Server([plan], max_batch=32, hbm_budget=2 * nbytes + 1)
    assert srv.info(0)[0] == 2
    srv.destroy()
    with pytest.raises(dh.DhError) as e:
        dh.Server([plan], max_batch=32, hbm_budget=nbytes - 1)
    assert e.value.code == dh.ERR_MEMORYALLOCATION
    plan.destroy()


def test_alignment_metric_goal_matches_oracle():
    """With a transfer-matrix metric as the goal and nothing to tweak, the
    goal is that metric of the oracle's coefficients at the plan's
    parameters; the report carries all nine (1024x1024, 2 pols, G=30)."""
    cfg = dh_synth.config(4)
    f, _ = dh_synth.make_frames(cfg, n_frames=3)
    p = cfg["truth"]
    oc = np.stack([oracle.process_frame(f[i].astype(np.float64), p)["coefs"] for i in range(f.shape[0])])
    for goal, indep, aa in (("IL", False, False), ("MDL", False, False), ("SNRMG", True, True)):
        ref = oracle.transfer_metrics(oc, 30, pol_independent=indep, mul_conj_trans=aa)
        _say("metric goal %s indep=%d aa=%d" % (goal, indep, aa))
        dh, plan, ft = _align_plan(p, f)
        plan.set_align_goal(goal, indep, aa)
        g = plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_TWEAK, what=0)
        rep = plan.align_report()
        plan.destroy()
        _say("goal gpu %.6f dB oracle %.6f dB" % (g, ref[goal]))
        assert rep.goal == oracle.METRICS.index(goal)
        assert abs(g - ref[goal]) <= 1e-3
        for i, k in enumerate(oracle.METRICS):
            if math.isinf(ref[k]):
                assert rep.metrics[i] == ref[k], k
            else:
                assert abs(rep.metrics[i] - ref[k]) <= 1e-3, (k, rep.metrics[i], ref[k])


def test_alignment_il_goal_recovers_truth():
    """AutoAlign on the insertion loss of the batch transfer matrix (each
    pol's tilt and defocus a coordinate of its own) finds the parameters the
    frames were made with; the report's metrics are those of the aligned
    plan's processed coefficients."""
    cfg = dh_synth.config(4)
    n = 20
    f, _ = dh_synth.make_frames(cfg, n_frames=n)
    truth = cfg["truth"]
    dh, plan, ft = _align_plan(cfg["params"], f)
    plan.set_align_goal("IL")
    _say("alignment on IL from nominal, %d frames" % n)
    g = plan.autoalign(ft, n, mode=dh.ALIGN_FULL, what=dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST, tol=1e-5)
    rep = plan.align_report()
    got = plan.params()
    bins = [1565e-9 / (512 * 20e-6) / oracle.DEG, 1565e-9 / (1024 * 20e-6) / oracle.DEG]
    _say("IL %.5f dB (after snap %.5f), %d trials, %d sweeps" % (g, rep.start_goal_db, rep.evaluations, rep.sweeps))
    for q in range(2):
        _say("pol %d tilt err %.3f / %.3f bins, defocus err %.4f D" % (
            q, (got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) / bins[0],
            (got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) / bins[1], got["defocus"][q] - truth["defocus"][q]))
    _say("waist err %.4f %%" % (100 * (got["waist"] / truth["waist"] - 1)))
    assert rep.goal == oracle.METRICS.index("IL") and g == pytest.approx(rep.metrics[0], abs=1e-4)
    for q in range(2):
        assert abs(got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) < 0.3 * bins[0]
        assert abs(got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) < 0.3 * bins[1]
        assert abs(got["defocus"][q] - truth["defocus"][q]) < 0.01
    assert abs(got["waist"] / truth["waist"] - 1) < 0.01
    plan.process(ft, n, None)
    after = plan.transfer_metrics()
    plan.destroy()
    for i, k in enumerate(oracle.METRICS):
        assert abs(after[k] - rep.metrics[i]) <= 1e-3, (k, after[k], rep.metrics[i])


def test_alignment_snap_centre_and_waist_match_oracle():
    """ESTIMATE on the beam centre and waist only: the intensity centroid and
    pooled second moment of the reconstructed fields, against the oracle's
    estimate from the same starting parameters (1024x1024, 2 pols, G=30)."""
    cfg = _half_height(dh_synth.config(4))
    f, _ = dh_synth.make_frames(cfg, n_frames=3)
    pix = 20e-6
    start = dict(cfg["truth"], beam_centre=[[1.7 * pix, -2.3 * pix], [-0.6 * pix, 0.8 * pix]],
                 waist=cfg["truth"]["waist"] * 1.1)
    ref_c, ref_w = oracle.snap_centre_waist(f, start)
    dh, plan, ft = _align_plan(start, f)
    _say("snap of centre and waist from an offset start")
    plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_ESTIMATE, what=dh.ALIGN_CENTRE | dh.ALIGN_WAIST)
    got = plan.params()
    rep = plan.align_report()
    plan.destroy()
    for q in range(2):
        for a in range(2):
            _say("pol %d axis %d centre gpu %.5f px oracle %.5f px" % (q, a, got["beam_centre"][q][a] / pix,
                                                                      ref_c[q][a] / pix))
            assert abs(got["beam_centre"][q][a] - ref_c[q][a]) < 1e-3 * pix
            assert rep.snap_centre[q][a] == got["beam_centre"][q][a]
    _say("waist gpu %.6e oracle %.6e" % (got["waist"], ref_w))
    assert abs(got["waist"] / ref_w - 1) < 1e-5 and rep.snap_waist == got["waist"]


def _half_height(cfg):
    """The 1024x1024 two-pol recipe with 512x512 FFT windows: room for the
    window to follow the beam centre (pol 0 to +x, pol 1 to -x, both in y)."""
    return dict(cfg, params=dict(cfg["params"], fft_h=512), truth=dict(cfg["truth"], fft_h=512))


def _bins(p):
    return [p["wavelength"] / (p["fft_w"] * p["pixel_size"]) / oracle.DEG,
            p["wavelength"] / (p["fft_h"] * p["pixel_size"]) / oracle.DEG]


def _shifted_centre_frames(n):
    cfg = _half_height(dh_synth.config(4))
    pix = 20e-6
    truth = dict(cfg["truth"], beam_centre=[[2.6 * pix, -1.4 * pix], [-3.2 * pix, 0.7 * pix]])
    f, _ = dh_synth.make_frames(dict(cfg, truth=truth), n_frames=n)
    return cfg, truth, f


def test_alignment_recovers_beam_centre():
    """FULL alignment of tilt, defocus, waist and beam centre from nominal, on
    frames whose beams sit off the nominal centres by whole and fractional
    pixels; the aligned plan then matches the oracle at its parameters."""
    cfg, truth, f = _shifted_centre_frames(20)
    n = f.shape[0]
    pix = 20e-6
    dh, plan, ft = _align_plan(cfg["params"], f)
    _say("alignment with beam centre from nominal, %d frames" % n)
    what = dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST | dh.ALIGN_CENTRE
    g = plan.autoalign(ft, n, mode=dh.ALIGN_FULL, what=what, tol=1e-5)
    rep = plan.align_report()
    got = plan.params()
    bins = _bins(truth)
    _say("goal %.5f dB (after snap %.5f), %d trials, %d sweeps; snap waist err %.2f %%" % (
        g, rep.start_goal_db, rep.evaluations, rep.sweeps, 100 * (rep.snap_waist / truth["waist"] - 1)))
    for q in range(2):
        _say("pol %d centre err %.3f / %.3f px (snap %.3f / %.3f), tilt err %.3f / %.3f bins, defocus err %.4f D" % (
            q, (got["beam_centre"][q][0] - truth["beam_centre"][q][0]) / pix,
            (got["beam_centre"][q][1] - truth["beam_centre"][q][1]) / pix,
            (rep.snap_centre[q][0] - truth["beam_centre"][q][0]) / pix,
            (rep.snap_centre[q][1] - truth["beam_centre"][q][1]) / pix,
            (got["tilt_deg"][q][0] - truth["tilt_deg"][q][0]) / bins[0],
            (got["tilt_deg"][q][1] - truth["tilt_deg"][q][1]) / bins[1], got["defocus"][q] - truth["defocus"][q]))
    _say("waist err %.4f %%" % (100 * (got["waist"] / truth["waist"] - 1)))
    for q in range(2):
        for a in range(2):
            assert abs(got["beam_centre"][q][a] - truth["beam_centre"][q][a]) < 0.1 * pix
            assert abs(rep.snap_centre[q][a] - truth["beam_centre"][q][a]) < 2.0 * pix
            assert abs(got["tilt_deg"][q][a] - truth["tilt_deg"][q][a]) < 0.3 * bins[a]
        assert abs(got["defocus"][q] - truth["defocus"][q]) < 0.01
    assert abs(got["waist"] / truth["waist"] - 1) < 0.01
    aligned = dict(truth, tilt_deg=got["tilt_deg"], defocus=got["defocus"], waist=got["waist"],
                   beam_centre=got["beam_centre"])
    plan.process(ft, n, None)
    coefs = plan.coefs(False)
    plan.destroy()
    for i in (0, n - 1):
        ref = oracle.process_frame(f[i].astype(np.float64), aligned)["coefs"]
        for pol in range(2):
            assert _rel(coefs[i][pol].astype(np.complex128), ref[pol]) <= TOL


def test_alignment_pol_lock():
    """Tilt and defocus locked across the polarisations: pol 1 carries pol 0's
    values after the alignment, which finds the common truth."""
    cfg = dh_synth.config(4)
    t0 = cfg["truth"]
    truth = dict(t0, tilt_deg=[t0["tilt_deg"][0], list(t0["tilt_deg"][0])], defocus=[t0["defocus"][0]] * 2)
    f, _ = dh_synth.make_frames(dict(cfg, truth=truth), n_frames=10)
    dh, plan, ft = _align_plan(cfg["params"], f)
    plan.set_pol_lock(dh.ALIGN_TILT | dh.ALIGN_DEFOCUS)
    with pytest.raises(dh.DhError):
        plan.set_pol_lock(dh.ALIGN_CENTRE)
    _say("alignment with locked tilt and defocus")
    plan.autoalign(ft, f.shape[0], mode=dh.ALIGN_FULL, what=dh.ALIGN_TILT | dh.ALIGN_DEFOCUS | dh.ALIGN_WAIST,
                   tol=1e-5)
    got = plan.params()
    plan.destroy()
    bins = [1565e-9 / (512 * 20e-6) / oracle.DEG, 1565e-9 / (1024 * 20e-6) / oracle.DEG]
    _say("tilt", got["tilt_deg"], "defocus", got["defocus"])
    assert got["tilt_deg"][1] == got["tilt_deg"][0] and got["defocus"][1] == got["defocus"][0]
    for a in range(2):
        assert abs(got["tilt_deg"][0][a] - truth["tilt_deg"][0][a]) < 0.3 * bins[a]
    assert abs(got["defocus"][0] - truth["defocus"][0]) < 0.01


# ---------------------------------------------------------------- IFFT mode 0 and the int16 format
@pytest.mark.parametrize("idx,cam,n,chunk", [
    (0, 0, 1, None),      # 128x128 G=4
    (1, 0, 7, 3),         # 640x512 2 pols G=9, ragged chunks
    (3, 1, 2, None),      # 640x512 uint16 G=9
    (4, 0, 2, None),      # 1024x1024 2 pols G=30
])
def test_mode0_coefficients_and_fields_vs_oracle(idx, cam, n, chunk):
    """IFFT mode 0: coefficients from the FFT-grid tables and the full-size
    fields made from the kept window, against the oracle in mode 0."""
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(idx, cam=cam, n=n)
    p = dict(cfg["params"], ifft_mode=0)
    _say("IFFT mode 0, recipe", idx, "camera", cam, f.shape)
    gpu = run_gpu(p, f, chunk=chunk)
    assert gpu["info"].path == dh.PATH_SPECTRAL
    assert gpu["field"].shape[2:] == (p["fft_h"], p["fft_w"])
    check_frames(p, f, gpu, range(n))


@pytest.mark.parametrize("idx,cam,n", [(1, 0, 3), (3, 2, 2)])
def test_mode0_without_decomposition(idx, cam, n):
    """IFFT mode 0 with G = 0: the field reconstruction alone (window and
    full-size fields, no coefficients) against the oracle."""
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(idx, cam=cam, n=n)
    p = dict(cfg["params"], ifft_mode=0, max_mg=0)
    _say("IFFT mode 0, G=0, recipe", idx, "camera", cam, f.shape)
    gpu = run_gpu(p, f)
    assert gpu["info"].path == dh.PATH_SPECTRAL and gpu["info"].modes == 0
    assert gpu["field"].shape[2:] == (p["fft_h"], p["fft_w"])
    check_frames(p, f, gpu, range(n))


def test_mode0_and_mode1_give_the_same_coefficients():
    """The two IFFT resolution modes are two quadratures of one overlap: on
    the GPU their coefficients agree as closely as the oracle's own modes."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(1, n=20)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    out = {}
    for mode in (1, 0):
        plan = dh.Plan(dict(cfg["params"], ifft_mode=mode), max_batch=20)
        plan.process(ft, 20, None)
        out[mode] = plan.coefs(True).astype(np.complex128)
        plan.destroy()
    worst = max(_rel(out[0][i][q], out[1][i][q]) for i in range(20) for q in range(2))
    _say("mode 0 vs mode 1 worst rel-L2 %.2e" % worst)
    assert worst <= 2e-6


def test_mode0_fields_across_export_groups():
    """1000 frames of 640x512 in IFFT mode 0 with fields: the export runs in
    groups of frames; sampled frames on both sides of each group edge."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg, pool, _ = _frames(1, n=50)
    n = 1000
    f = dh_synth.tile_pool(pool, n)
    p = dict(cfg["params"], ifft_mode=0, keep_fields=1)
    plan = dh.Plan(p, max_batch=n)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    _say("mode-0 fields, batch %d" % n)
    plan.process(ft, n, None)
    fields = plan.fields()
    coefs = plan.coefs(False)
    plan.destroy()
    for i in (0, 296, 297, 593, 594, 999):
        ref = oracle.process_frame(f[i].astype(np.float64), p)
        for q in range(2):
            assert _rel(fields[i][q].astype(np.complex128), ref["field"][q]) <= TOL, (i, q)
            assert _rel(coefs[i][q].astype(np.complex128), ref["coefs"][q]) <= TOL, (i, q)


def test_int16_conversion_is_bit_exact():
    """dh_fields_to_int16 on seeded synthetic fields (ragged length, a zero
    field, values planted on rounding ties) against the oracle's FP32
    conversion: every code and scale identical."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    rng = np.random.default_rng(20240417)
    n, length = 5, 4099
    f = (rng.normal(size=(n, length)) + 1j * rng.normal(size=(n, length))).astype(np.complex64)
    f[1] *= np.float32(1e-3)
    f[2] = 0
    f[3, :8] = np.array([32767.0, 2.5, 3.5, -2.5, -3.5, 0.5, 1.5, -0.5], dtype=np.float32)   # scale 1: ties
    f[3, 8:] = (f[3, 8:] * np.float32(100)).astype(np.complex64)
    dev = torch.from_numpy(f).cuda()
    re = torch.empty((n, length), dtype=torch.int16, device="cuda")
    im = torch.empty_like(re)
    sc = torch.empty(n, dtype=torch.float32, device="cuda")
    dh.fields_to_int16(dev, n, length, re, im, sc)
    torch.cuda.synchronize()
    gre, gim, gsc = re.cpu().numpy(), im.cpu().numpy(), sc.cpu().numpy()
    for e in range(n):
        ore, oim, osc = oracle.fields_to_int16(f[e])
        _say("field %d scale gpu %r oracle %r" % (e, float(gsc[e]), float(osc)))
        assert gsc[e] == osc
        assert np.array_equal(gre[e], ore) and np.array_equal(gim[e], oim)


def test_plan_fields16_match_oracle_fields():
    """The plan's int16 export of its fields: codes within one step of the
    oracle's conversion of the oracle's field (the two FP32 fields differ by
    rounding), the decoded field within half a step plus that rounding."""
    import paper_2204_02348_amd as dh
    torch = _torch()
    for mode in (1, 0):
        cfg, f, _ = _frames(1, n=3)
        p = dict(cfg["params"], ifft_mode=mode, keep_fields=1)
        plan = dh.Plan(p, max_batch=3)
        ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
        plan.process(ft, 3, None)
        re, im, sc = plan.fields16()
        plan.destroy()
        _say("fields16 mode %d shape %s" % (mode, re.shape))
        for i in range(3):
            ref = oracle.process_frame(f[i].astype(np.float64), p)["field"]
            for q in range(2):
                ore, oim, osc = oracle.fields_to_int16(ref[q])
                assert abs(float(sc[i, q]) / float(osc) - 1) < 1e-5
                assert np.abs(re[i, q].astype(np.int32) - ore).max() <= 1
                assert np.abs(im[i, q].astype(np.int32) - oim).max() <= 1
                dec = (re[i, q] + 1j * im[i, q].astype(np.float64)) / float(sc[i, q])
                step = 1.0 / float(sc[i, q])
                assert np.abs(dec - ref[q]).max() <= 0.5 * step + 1e-5 * np.abs(ref[q]).max()


# ---------------------------------------------------------------- basis transforms (LG, custom)
def _basis_run(p, f, basis, matrix=None, chunk=None):
    torch = _torch()
    import paper_2204_02348_amd as dh
    if chunk:
        os.environ["DH_CHUNK_FRAMES"] = str(chunk)
    try:
        plan = dh.Plan(p, max_batch=f.shape[0])
    finally:
        os.environ.pop("DH_CHUNK_FRAMES", None)
    plan.set_basis(basis, matrix)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    plan.process(ft, f.shape[0], None)
    out = plan.coefs(False), plan.coefs(True), plan.transfer_metrics()
    plan.destroy()
    return out


@pytest.mark.parametrize("idx,n,chunk", [(1, 7, 3), (4, 2, None)])
def test_lg_basis_vs_oracle(idx, n, chunk):
    """LG coefficients (raw and normalised) against the oracle's HG
    coefficients times its HG->LG transform (exact Gauss-Hermite overlaps)."""
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(idx, n=n)
    p = cfg["params"]
    raw, nrm, met = _basis_run(p, f, dh.BASIS_LG, chunk=chunk)
    t = oracle.hg_to_lg(p["max_mg"])
    _say("LG basis, recipe %d, %d frames" % (idx, n))
    oc = []
    for i in range(n):
        ref = oracle.process_frame(f[i].astype(np.float64), p)
        oc.append(ref["coefs"])
        lr, ln = oracle.apply_basis(ref["coefs"], t), oracle.apply_basis(ref["coefs_norm"], t)
        for q in range(2):
            assert _rel(raw[i][q].astype(np.complex128), lr[q]) <= TOL
            assert _rel(nrm[i][q].astype(np.complex128), ln[q]) <= TOL
    ref = oracle.transfer_metrics(oracle.apply_basis(np.stack(oc), t), p["max_mg"])
    for k in oracle.METRICS:
        assert abs(met[k] - ref[k]) <= 1e-3, (k, met[k], ref[k])


def test_custom_basis_vs_oracle():
    """A seeded 17 x 60 custom matrix on a G=9 plan (45 HG modes: columns 45..59
    unused): coefficients and metrics (each output mode its own group)."""
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(1, n=5)
    p = cfg["params"]
    rng = np.random.default_rng(99)
    m = (rng.normal(size=(17, 60)) + 1j * rng.normal(size=(17, 60))).astype(np.complex64)
    raw, nrm, met = _basis_run(p, f, dh.BASIS_CUSTOM, m)
    t = oracle.custom_transform(m.astype(np.complex128), oracle.mode_count(p["max_mg"]))
    _say("custom basis 17 x 60, shape", raw.shape)
    assert raw.shape == (5, 2, 17)
    oc = []
    for i in range(5):
        ref = oracle.process_frame(f[i].astype(np.float64), p)
        oc.append(ref["coefs"])
        lr, ln = oracle.apply_basis(ref["coefs"], t), oracle.apply_basis(ref["coefs_norm"], t)
        for q in range(2):
            assert _rel(raw[i][q].astype(np.complex128), lr[q]) <= TOL
            assert _rel(nrm[i][q].astype(np.complex128), ln[q]) <= TOL
    ref = oracle.transfer_metrics(oracle.apply_basis(np.stack(oc), t), p["max_mg"], groups=np.arange(17))
    for k in oracle.METRICS:
        assert abs(met[k] - ref[k]) <= 1e-3, (k, met[k], ref[k])


def test_serving_returns_the_basis_coefficients():
    """A camera whose plan has the LG basis: each served result equals the
    plan's own LG coefficients of that frame, bit for bit."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(3, 1)
    f, _ = dh_synth.make_frames(cfg, n_frames=8)
    plan = dh.Plan(cfg["params"], max_batch=8)
    plan.set_basis(dh.BASIS_LG)
    pool = torch.from_numpy(f).cuda()
    srv = dh.Server([plan], max_batch=8, hbm_budget=4 << 30)
    per = srv.info(0)[2]
    assert per == oracle.mode_count(cfg["params"]["max_mg"])
    n = 40
    t = np.linspace(0.0, 2e-3, n)
    cam = np.zeros(n, dtype=np.int32)
    idx = np.arange(n) % 8
    res = [np.zeros(per, dtype=np.complex64) for _ in range(n)]
    torch.cuda.synchronize()
    srv.replay(t, cam, [pool[i].data_ptr() for i in idx], res)
    srv.destroy()
    _say("served %d LG results" % n)
    for i in range(8):
        plan.process(pool[i], 1, None)
        alone = plan.coefs(True)[0].reshape(-1)
        for k in np.nonzero(idx == i)[0]:
            assert np.array_equal(res[k], alone), (i, k)
    plan.destroy()


# ---------------------------------------------------------------- wavelength sweeps and averaging
def _sweep_run(p, f, n_out, lams=None, in_order=0, out_order=0, avg=1, mode=0, chunk=None):
    torch = _torch()
    import paper_2204_02348_amd as dh
    if chunk:
        os.environ["DH_CHUNK_FRAMES"] = str(chunk)
    try:
        plan = dh.Plan(p, max_batch=f.shape[0])
    finally:
        os.environ.pop("DH_CHUNK_FRAMES", None)
    if lams is not None:
        plan.set_wavelengths(lams, in_order, out_order)
    if avg > 1:
        plan.set_averaging(avg, mode)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.process(ft, n_out, s)
    out = dict(coefs=plan.coefs(False), coefs_norm=plan.coefs(True))
    if p.get("keep_window"):
        out["window"] = plan.window()
    if p.get("keep_fields"):
        out["field"] = plan.fields()
    torch.cuda.synchronize()
    plan.destroy()
    return out


def _check_sweep(gpu, ref, keys, tol=TOL):
    worst = {}
    for k in keys:
        for o in range(ref[k].shape[0]):
            for q in range(ref[k].shape[1]):
                worst[k] = max(worst.get(k, 0.0), _rel(gpu[k][o][q].astype(np.complex128), ref[k][o][q]))
    _say("worst rel-L2", {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("in_order,out_order", [(0, 0), (0, 1), (1, 0)])
def test_wavelength_sweep_vs_oracle(in_order, out_order):
    """Three wavelengths, two inputs, 640x512 two pols G=9 on the field path
    with windows and fields, against the oracle's per-frame wavelengths."""
    cfg, f, _ = _frames(1, n=6)
    p = dict(cfg["params"], keep_window=1, keep_fields=1)
    lams = [1565e-9 * 0.99, 1565e-9, 1565e-9 * 1.012]
    _say("sweep in_order %d out_order %d" % (in_order, out_order))
    gpu = _sweep_run(p, f, 6, lams, in_order, out_order, chunk=4)
    ref = oracle.process_sweep(f.astype(np.float64), p, lams, in_order=in_order, out_order=out_order)
    _check_sweep(gpu, ref, ("coefs", "coefs_norm", "window", "field"))


@pytest.mark.parametrize("mode", [0, 1])
def test_averaging_vs_oracle(mode):
    """Three outputs, each the phase-aligned average of three frames
    (sequential or interlaced), over chunks of four frames."""
    cfg, f, _ = _frames(1, n=9)
    p = dict(cfg["params"], keep_window=1, keep_fields=1)
    _say("averaging mode %d" % mode)
    gpu = _sweep_run(p, f, 3, avg=3, mode=mode, chunk=4)
    ref = oracle.process_sweep(f.astype(np.float64), p, [p["wavelength"]], avg_count=3, avg_mode=mode)
    _check_sweep(gpu, ref, ("coefs", "coefs_norm", "window", "field"))


def test_averaged_sweep_spectral_and_mode0():
    """Two wavelengths, averaging over sequential sweeps: on the spectral path
    (coefficients only), and in IFFT mode 0 with the fields exported."""
    cfg, f, _ = _frames(1, n=8)
    lams = [1565e-9 * 1.008, 1565e-9 * 0.994]
    for extra in (dict(), dict(ifft_mode=0, keep_fields=1)):
        p = dict(cfg["params"], **extra)
        _say("averaged sweep", extra)
        gpu = _sweep_run(p, f, 4, lams, 0, 1, avg=2, mode=2)
        ref = oracle.process_sweep(f.astype(np.float64), p, lams, avg_count=2, avg_mode=2, in_order=0, out_order=1)
        _check_sweep(gpu, ref, ("coefs", "coefs_norm") + (("field",) if extra else ()))


def test_sweep_with_lg_basis_metrics_and_int16_fields():
    """A 2-wavelength sweep (slow out) averaged over 2 interlaced repetitions,
    in the LG basis, with fields: LG coefficients, the transfer-matrix metrics
    of the LG matrix, and the int16 fields, against the oracle."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(1, n=8)
    p = dict(cfg["params"], keep_fields=1)
    lams = [1565e-9 * 0.995, 1565e-9 * 1.004]
    plan = dh.Plan(p, max_batch=8)
    plan.set_wavelengths(lams, dh.WL_FAST, dh.WL_SLOW)
    plan.set_averaging(2, dh.AVG_INTERLACED)
    plan.set_basis(dh.BASIS_LG)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    plan.process(ft, 4, None)
    raw, nrm = plan.coefs(False), plan.coefs(True)
    met = plan.transfer_metrics()
    re, im, sc = plan.fields16()
    plan.destroy()
    ref = oracle.process_sweep(f.astype(np.float64), p, lams, avg_count=2, avg_mode=1, in_order=0, out_order=1)
    t = oracle.hg_to_lg(p["max_mg"])
    _say("sweep + averaging + LG + int16")
    for o in range(4):
        for q in range(2):
            assert _rel(raw[o][q].astype(np.complex128), oracle.apply_basis(ref["coefs"][o], t)[q]) <= TOL
            assert _rel(nrm[o][q].astype(np.complex128), oracle.apply_basis(ref["coefs_norm"][o], t)[q]) <= TOL
            ore, oim, osc = oracle.fields_to_int16(ref["field"][o][q])
            assert abs(float(sc[o, q]) / float(osc) - 1) < 1e-5
            assert np.abs(re[o, q].astype(np.int32) - ore).max() <= 1
            assert np.abs(im[o, q].astype(np.int32) - oim).max() <= 1
    mref = oracle.transfer_metrics(oracle.apply_basis(ref["coefs"], t), p["max_mg"])
    for k in oracle.METRICS:
        assert abs(met[k] - mref[k]) <= 1e-3, (k, met[k], mref[k])


def test_sweep_rejections():
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg, f, _ = _frames(1, n=4)
    plan = dh.Plan(cfg["params"], max_batch=4)
    plan.set_wavelengths([1565e-9, 1566e-9, 1567e-9])
    ft = torch.from_numpy(f).cuda()
    with pytest.raises(dh.DhError) as e:
        plan.process(ft, 4, None)                       # not a whole number of sweeps
    assert e.value.code == dh.ERR_INVALIDDIMENSION
    plan.set_wavelengths([])
    plan.set_averaging(3)
    ft6 = torch.cat([ft, ft[:2]])                       # the frames the call reads
    with pytest.raises(dh.DhError) as e:
        plan.process(ft6, 2, None)                      # 6 staged frames > max_batch 4
    assert e.value.code == dh.ERR_INVALIDDIMENSION
    with pytest.raises(dh.DhError):
        plan.autoalign(ft, 1)
    with pytest.raises(dh.DhError):
        dh.Server([plan], max_batch=4)
    with pytest.raises(dh.DhError) as e:
        plan.set_wavelengths([1565e-9, -1.0])
    assert e.value.code == dh.ERR_INVALIDARGUMENT
    plan.destroy()


# ---------------------------------------------------------------- transfer-matrix metrics
@pytest.mark.parametrize("n", [90, 1000])
def test_transfer_metrics_match_oracle(n):
    """The nine metrics of the batch transfer matrix (640x512, 2 pols, G=9:
    90 columns) on the GPU, against the oracle's metrics of the same
    coefficients (both FP64) for every option, and against the oracle's own
    coefficients for the default options."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg, pool, _ = _frames(1, n=min(n, 90))
    f = dh_synth.tile_pool(pool, n) if n > 90 else pool
    plan = dh.Plan(cfg["params"], max_batch=n)
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    plan.process(ft, n, None)
    coefs = plan.coefs(False).astype(np.complex128)
    got = {}
    for indep in (False, True):
        for aa in (False, True):
            got[(indep, aa)] = plan.transfer_metrics(indep, aa)
    plan.destroy()
    for (indep, aa), g in got.items():
        ref = oracle.transfer_metrics(coefs, 9, pol_independent=indep, mul_conj_trans=aa)
        _say("metrics n=%d indep=%d aa=%d" % (n, indep, aa), {k: "%.6f" % v for k, v in g.items()})
        for k in oracle.METRICS:
            if math.isinf(ref[k]):
                assert g[k] == ref[k], (indep, aa, k)
            else:
                assert abs(g[k] - ref[k]) <= 1e-6, (indep, aa, k, g[k], ref[k])
    if n == 90:
        oc = np.stack([oracle.process_frame(f[i].astype(np.float64), cfg["params"])["coefs"] for i in range(n)])
        ref = oracle.transfer_metrics(oc, 9)
        for k in oracle.METRICS:
            assert abs(got[(False, False)][k] - ref[k]) <= 1e-3, k
