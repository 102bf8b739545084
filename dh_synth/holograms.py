"""Synthetic holograms shaped like the paper's workloads.

Forward model (Background, "off-axis digital holography"): a signal field S
that is a sum of Hermite-Gaussian modes, a tilted (and optionally defocused)
plane-wave reference R = A exp(i phi_R), and the camera records |S + R|^2,
scaled to 12-bit counts, optionally with Poisson shot noise and Gaussian read
noise. Two polarisations occupy the left and right halves of the frame.

This module evaluates the HG modes from the closed form with explicit
(physicists') Hermite polynomials via numpy.polynomial.hermite, a route that is
independent of the normalised recurrence used elsewhere.

Seeds: numpy PCG64 from SeedSequence(BASE_SEED + config index); the config
draws come from the first child sequence, frame i from child i of the second.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import hermite as _herm

BASE_SEED = 220402348
_PIX = 20e-6
_LAM = 1565e-9
_WMAX_DEG = _LAM / (2 * _PIX) * 180.0 / math.pi
_RADIUS_DEG = 0.32 * _WMAX_DEG


def hg_closed_form(n: int, x: np.ndarray, waist: float) -> np.ndarray:
    """u_n(x) = (2/pi)^(1/4) (2^n n! w)^(-1/2) H_n(sqrt2 x/w) exp(-x^2/w^2)."""
    x = np.asarray(x, dtype=np.float64)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    lognorm = 0.25 * math.log(2 / math.pi) - 0.5 * (n * math.log(2) + math.lgamma(n + 1) + math.log(waist))
    s = math.sqrt(2.0) * x / waist
    return _herm.hermval(s, coef) * np.exp(lognorm - x * x / (waist * waist))


def _modes(group_count):
    out = []
    for g in range(group_count):
        for m in range(g, -1, -1):
            out.append((m, g - m))
    return out


def _base_params(frame_w, frame_h, pols, fft_w, fft_h, waist, groups, dtype="f32"):
    return dict(frame_w=frame_w, frame_h=frame_h, pol_count=pols, fft_w=fft_w, fft_h=fft_h,
                pixel_size=_PIX, wavelength=_LAM,
                beam_centre=[[0.0, 0.0], [0.0, 0.0]],
                window_radius_deg=_RADIUS_DEG,
                tilt_deg=[[1.5, 1.5], [1.5, 1.5]], defocus=[0.0, 0.0],
                waist=waist, max_mg=groups, input_dtype=dtype)


def config(idx: int, camera: int = 0) -> dict:
    """Workload recipe `idx` (0..4) as a dict with 'params' (what a plan is
    built from), 'truth' (the parameters the holograms are synthesised with),
    'frames', 'noise' and 'dtype'. For idx 3, `camera` picks one of the four
    serving cameras."""
    ss = np.random.SeedSequence(BASE_SEED + idx)
    cfg_ss, _ = ss.spawn(2)
    rng = np.random.Generator(np.random.PCG64(cfg_ss))
    if idx == 0:      # 1 frame 128x128, 1 pol, 10 modes, 12-bit, no noise
        p = _base_params(128, 128, 1, 128, 128, 200e-6, 4)
        c = dict(params=p, frames=1, noise=False)
    elif idx == 1:    # 1000 frames 640x512, 2 pols, G=9, defocus +-0.05 D, shot+read noise
        p = _base_params(640, 512, 2, 320, 512, 400e-6, 9)
        p["defocus"] = [float(d) for d in rng.uniform(-0.05, 0.05, size=2)]
        c = dict(params=p, frames=1000, noise=True)
    elif idx == 2:    # config 0 with G=20 (210 modes)
        p = _base_params(128, 128, 1, 128, 128, 200e-6, 20)
        c = dict(params=p, frames=1, noise=False)
    elif idx == 3:    # serving cameras, uint16, one pol each
        cams = [(320, 256, 5, 300e-6), (640, 512, 9, 400e-6),
                (1024, 1024, 15, 600e-6), (2048, 2048, 20, 1e-3)]
        w, h, gcount, waist = cams[camera]
        p = _base_params(w, h, 1, w, h, waist, gcount, dtype="u16")
        c = dict(params=p, frames=64, noise=True)
    elif idx == 4:    # alignment workload 1024^2, 2 pols, G=30, unknown tilt/defocus/waist
        p = _base_params(1024, 1024, 2, 512, 1024, 500e-6, 30)
        c = dict(params=p, frames=50, noise=True)
        truth = dict(p)
        truth["tilt_deg"] = [[1.5 + float(t) for t in rng.uniform(-0.3, 0.3, size=2)] for _ in range(2)]
        truth["defocus"] = [float(d) for d in rng.uniform(-0.2, 0.2, size=2)]
        truth["waist"] = 500e-6 * (1.0 + float(rng.uniform(-0.2, 0.2)))
        c["truth"] = truth
    else:
        raise ValueError(idx)
    c.setdefault("truth", dict(c["params"]))
    c["dtype"] = c["params"]["input_dtype"]
    c["index"] = idx
    c["camera"] = camera
    return c


def _plane_cache(truth: dict) -> list:
    """Per-pol coordinate axes, HG tables and reference-phase factors, which
    every frame of a recipe shares."""
    fw, fh, npol = truth["frame_w"], truth["frame_h"], truth["pol_count"]
    pix, lam, waist = truth["pixel_size"], truth["wavelength"], truth["waist"]
    half = fw // npol
    modes = _modes(truth["max_mg"])
    gmax = max(max(m, n) for m, n in modes) + 1 if modes else 0
    out = []
    for pol in range(npol):
        bcx, bcy = truth["beam_centre"][pol]
        x = (np.arange(half) - half // 2) * pix - bcx
        y = (np.arange(fh) - fh // 2) * pix - bcy
        hx = np.stack([hg_closed_form(m, x, waist) for m in range(gmax)]) if gmax else None
        hy = np.stack([hg_closed_form(n, y, waist) for n in range(gmax)]) if gmax else None
        tx, ty = (t * math.pi / 180.0 for t in truth["tilt_deg"][pol])
        d = truth["defocus"][pol]
        phi = (2 * math.pi * (tx * x[None, :] + ty * y[:, None]) / lam
               + math.pi * d * (x[None, :] ** 2 + y[:, None] ** 2) / lam)
        out.append(dict(hx=hx, hy=hy, gmax=gmax, cos=np.cos(phi), sin=np.sin(phi)))
    return out


def forward_hologram(truth: dict, coefs: np.ndarray, cache: list | None = None) -> np.ndarray:
    """|S_p + R_p|^2 on every pixel of the frame (FP64, before scaling).

    coefs: [pol][mode] complex, modes ordered by group ascending then m
    descending. The reference amplitude is A = max |S| over the frame. The
    reference phase is 2 pi (theta_x x + theta_y y)/lambda + pi D (x^2+y^2)/lambda,
    with x, y measured from the pol's beam centre (in metres relative to the
    centre pixel of its half-frame)."""
    fw, fh, npol = truth["frame_w"], truth["frame_h"], truth["pol_count"]
    half = fw // npol
    modes = _modes(truth["max_mg"])
    if cache is None:
        cache = _plane_cache(truth)
    sig = []
    for pol in range(npol):
        c = cache[pol]
        g = c["gmax"]
        if g:
            cmat = np.zeros((g, g), dtype=np.complex128)
            for k, (m, n) in enumerate(modes):
                cmat[n, m] = coefs[pol][k]
            sig.append(c["hy"].T @ cmat @ c["hx"])
        else:
            sig.append(np.zeros((fh, half), dtype=np.complex128))
    amp = max(float(np.abs(s).max()) for s in sig)
    frame = np.empty((fh, fw), dtype=np.float64)
    for pol, s in enumerate(sig):
        c = cache[pol]
        re = s.real + amp * c["cos"]
        im = s.imag + amp * c["sin"]
        frame[:, pol * half:(pol + 1) * half] = re * re + im * im
    return frame


def _frame_job(args):
    cfg, kid, quantise, nm, cache = args
    truth = cfg["truth"]
    npol = truth["pol_count"]
    rng = np.random.Generator(np.random.PCG64(kid))
    c = (rng.standard_normal((npol, nm)) + 1j * rng.standard_normal((npol, nm))) / math.sqrt(2)
    pw = float(np.sum(np.abs(c) ** 2))
    c = c / math.sqrt(pw) if pw > 0 else c
    f = forward_hologram(truth, c, cache)
    if not quantise:
        return f, c
    level = 4095.0 * f / f.max()
    if cfg["noise"]:
        level = rng.poisson(0.9 * level).astype(np.float64) + rng.normal(0.0, 2.0, size=level.shape)
    out_dtype = np.uint16 if cfg["dtype"] == "u16" else np.float32
    return np.clip(np.rint(level), 0, 4095).astype(out_dtype), c


def make_frames(cfg: dict, n_frames: int | None = None, quantise: bool = True,
                first: int = 0, workers: int = 1):
    """Frames i = first .. first+n-1 of recipe `cfg`: (frames, coefs).

    frames: [n][frame_h][frame_w], float32 (or uint16 for u16 recipes; FP64
    when quantise is False); coefs: [n][pol][mode] complex128 true
    coefficients, unit power per frame over both pols. workers > 1 uses a
    thread pool; the frames do not depend on it."""
    truth = cfg["truth"]
    n = cfg["frames"] if n_frames is None else n_frames
    ss = np.random.SeedSequence(BASE_SEED + cfg["index"] + 1000 * cfg.get("camera", 0))
    _, frames_ss = ss.spawn(2)
    kids = frames_ss.spawn(first + n)[first:]
    nm = len(_modes(truth["max_mg"]))
    npol = truth["pol_count"]
    out_dtype = np.float64 if not quantise else (np.uint16 if cfg["dtype"] == "u16" else np.float32)
    frames = np.empty((n, truth["frame_h"], truth["frame_w"]), dtype=out_dtype)
    coefs = np.empty((n, npol, nm), dtype=np.complex128)
    cache = _plane_cache(truth)
    if workers > 1 and n > 1:
        # threads, not processes: safe in a process that already holds a GPU
        # context (numpy releases the GIL in the large array operations)
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for i, (f, c) in enumerate(ex.map(lambda kid: _frame_job((cfg, kid, quantise, nm, cache)), kids)):
                frames[i], coefs[i] = f, c
    else:
        for i, kid in enumerate(kids):
            frames[i], coefs[i] = _frame_job((cfg, kid, quantise, nm, cache))
    return frames, coefs


def tile_pool(pool: np.ndarray, n: int) -> np.ndarray:
    """Repeat a pool of distinct frames up to n frames (frame i = pool[i % len])."""
    reps = -(-n // pool.shape[0])
    return np.concatenate([pool] * reps, axis=0)[:n]
