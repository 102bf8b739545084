"""Plain FP64 oracle of the per-frame off-axis holography pipeline.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

What it computes follows the paper (digHolo User Guide, arXiv 2204.02348):

* Background, "off-axis digital holography": the camera records |S+R|^2; the
  Fourier transform of the SR* cross term is the signal spectrum shifted by
  the reference angle; selecting it, transforming back and removing the
  reference tilt gives the signal field.
* Background, "How do you choose the angle of the Reference Field?": the
  maximum resolvable angle is w_max = lambda / (2 * pixel) and the Fourier
  window radius w_c is a fraction of it.
* Background, "digHolo processing pipeline", steps 1-3: window + FFT, window
  select + IFFT + tilt removal with the field centred on the beam centre,
  then a Hermite-Gaussian modal decomposition.
* API sections "Window sizes" (FourierWindowRadius, IFFT resolution mode 1),
  "Alignment" (tilt in degrees, defocus in dioptre, beam centre, one waist
  shared by both polarisations) and "Modal basis" (HG(m,n) with m+n <
  groupCount; coefficients laid out batch x (pol x mode), pol blocks).

The pipeline produces, per frame and polarisation, a result with a plain
definition, so the oracle writes that definition out directly, with no FFT
factorisation, blocking or reordering:

  spectrum   I~(u,v) = sum_j I[j] exp(-2 pi i (u x_j/(Nx p) + v y_j/(Ny p)))
             (explicit DFT matrices at the needed bins; x_j, y_j in metres
             relative to the beam centre)
  window     M(u,v) I~(u,v), M = 1 inside the ellipse of radius r (in bins)
             centred on the SR* term at bins (-a_x, -a_y)
  field      E(x',y') = exp(i phi_R(x',y')) / (Nx Ny)
                        * sum_{u,v} M I~ exp(2 pi i (u x'/(Nx p) + v y'/(Ny p)))
             on the coarse grid x'_k = (k - Wx/2) p', p' = Nx p / Wx
  reference  phi_R = 2 pi (a_x x/(Nx p) + a_y y/(Ny p)) + pi D (x^2+y^2)/lambda
  coefs      c_mn = sum_{k,l} E(x'_k,y'_l) u_m(x'_k) u_n(y'_l) p'_x p'_y
  norm       c_hat = c / sqrt(sum over both pols and all modes of |c|^2)

Where the paper is silent or garbled, the readings taken are the ones written
out above and in the functions below (window ratio and IFFT size rule,
paraxial angle -> bin mapping, which cross term, defocus sign, coordinate
origins, mask boundary, normalisations, mode ordering, beam-centre origin).
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


# --------------------------------------------------------------------------
# geometry (Background: "How do you choose the angle of the Reference Field?";
# "Window sizes": FourierWindowRadius; "Alignment": tilt, beam centre)
# --------------------------------------------------------------------------
def w_max_rad(pixel: float, lam: float) -> float:
    """Maximum resolvable angle set by the pixel pitch, lambda / (2 pixel)."""
    return lam / (2.0 * pixel)


def tilt_bins(tilt_deg: float, n: int, pixel: float, lam: float) -> float:
    """Position of the cross term along one axis, in FFT bins (paraxial:
    an angle theta is the spatial frequency theta/lambda; bin u is the
    frequency u/(N p))."""
    return tilt_deg * DEG * n * pixel / lam


def radius_bins(radius_deg: float, n: int, pixel: float, lam: float) -> float:
    """Fourier window radius in bins along an axis of n samples: w_max maps
    to the Nyquist bin n/2."""
    return (radius_deg * DEG / w_max_rad(pixel, lam)) * (n / 2.0)


def _prime_factors_le_13(n: int) -> bool:
    for f in (2, 3, 5, 7, 11, 13):
        while n % f == 0:
            n //= f
    return n == 1


def ifft_size(r_bins: float) -> int:
    """IFFT length (IFFT resolution mode 1, the Fourier-window size): the
    smallest multiple of 16 with no prime factor above 13 that holds every
    bin of a window of radius r_bins, i.e. >= floor(2 r) + 1."""
    need = int(math.floor(2.0 * r_bins)) + 1
    w = 16
    while w < need or not _prime_factors_le_13(w):
        w += 16
    return w


def mode_list(group_count: int):
    """HG(m,n) with m+n < groupCount ("Modal basis"); order: group g = m+n
    ascending, inside a group m descending."""
    out = []
    for g in range(group_count):
        for m in range(g, -1, -1):
            out.append((m, g - m))
    return out


def mode_count(group_count: int) -> int:
    return len(mode_list(group_count))


def window_origin(params: dict, pol: int):
    """Pixel origin (x0, y0) of the FFT window of `pol` and the sub-pixel
    remainder (dx, dy) in metres of its beam centre.

    Two polarisations sit on opposite halves of the frame width (pipeline
    step 1). The beam centre of a pol is given in metres relative to the
    centre pixel of its half-frame (pixel index half/2); the window is cut
    so that its pixel N/2 is the beam-centre pixel nearest to the centre.
    """
    fw, fh = params["frame_w"], params["frame_h"]
    npol = params["pol_count"]
    nx, ny = params["fft_w"], params["fft_h"]
    p = params["pixel_size"]
    half = fw // npol
    bcx, bcy = params["beam_centre"][pol]
    ix = int(math.floor(bcx / p + 0.5))
    iy = int(math.floor(bcy / p + 0.5))
    x0 = pol * half + half // 2 + ix - nx // 2
    y0 = fh // 2 + iy - ny // 2
    dx = bcx - ix * p
    dy = bcy - iy * p
    return x0, y0, dx, dy


def mask_bins(ax, ay, rx, ry, us, vs):
    """Circular (in angle; elliptical in bins when Nx != Ny) Fourier window
    around the SR* term at (-ax, -ay), boundary included. Boolean [v][u]."""
    uu = np.asarray(us, dtype=np.float64)[None, :]
    vv = np.asarray(vs, dtype=np.float64)[:, None]
    return ((uu + ax) / rx) ** 2 + ((vv + ay) / ry) ** 2 <= 1.0


def geometry(params: dict) -> dict:
    """Everything the definition needs, per polarisation, in FP64."""
    nx, ny = params["fft_w"], params["fft_h"]
    p, lam = params["pixel_size"], params["wavelength"]
    rx = radius_bins(params["window_radius_deg"], nx, p, lam)
    ry = radius_bins(params["window_radius_deg"], ny, p, lam)
    wx, wy = ifft_size(rx), ifft_size(ry)
    pols = []
    for pol in range(params["pol_count"]):
        ax = tilt_bins(params["tilt_deg"][pol][0], nx, p, lam)
        ay = tilt_bins(params["tilt_deg"][pol][1], ny, p, lam)
        # every bin of the lattice that can lie inside the window
        us = np.arange(int(math.floor(-ax - rx)) - 1, int(math.ceil(-ax + rx)) + 2)
        vs = np.arange(int(math.floor(-ay - ry)) - 1, int(math.ceil(-ay + ry)) + 2)
        m = mask_bins(ax, ay, rx, ry, us, vs)
        x0, y0, dx, dy = window_origin(params, pol)
        pols.append(dict(ax=ax, ay=ay, us=us, vs=vs, mask=m, x0=x0, y0=y0,
                         dx=dx, dy=dy, defocus=params["defocus"][pol]))
    # the reconstructed field's grid: IFFT resolution mode 1 (the window
    # size, pitch N p / W) or mode 0 (the FFT size, the camera pitch)
    mode = params.get("ifft_mode", 1)
    if mode not in (0, 1):
        raise ValueError("ifft_mode is 0 or 1")
    fx, fy = (wx, wy) if mode == 1 else (nx, ny)
    return dict(nx=nx, ny=ny, p=p, lam=lam, rx=rx, ry=ry, wx=wx, wy=wy,
                px2=nx * p / fx, py2=ny * p / fy, fx=fx, fy=fy, ifft_mode=mode, pols=pols)


# --------------------------------------------------------------------------
# Hermite-Gaussian basis ("Modal basis": HG modes of one waist)
# --------------------------------------------------------------------------
def hermite_gauss_1d(n_max: int, x: np.ndarray, waist: float) -> np.ndarray:
    """u_n(x) for n < n_max, unit L2 norm, w = 1/e^2 intensity radius.

    u_n(x) = 2^(1/4) w^(-1/2) psi_n(sqrt(2) x / w), with the normalised
    Hermite functions psi_0(s) = pi^(-1/4) exp(-s^2/2),
    psi_{n+1} = sqrt(2/(n+1)) s psi_n - sqrt(n/(n+1)) psi_{n-1}.
    Returns [n_max][len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    s = math.sqrt(2.0) * x / waist
    out = np.zeros((max(n_max, 0), x.size), dtype=np.float64)
    if n_max <= 0:
        return out
    psi_prev = np.zeros_like(s)
    psi = math.pi ** -0.25 * np.exp(-0.5 * s * s)
    out[0] = psi
    for n in range(0, n_max - 1):
        nxt = math.sqrt(2.0 / (n + 1)) * s * psi - math.sqrt(n / (n + 1)) * psi_prev
        psi_prev, psi = psi, nxt
        out[n + 1] = psi
    return out * (2.0 ** 0.25 / math.sqrt(waist))


# --------------------------------------------------------------------------
# the pipeline, as definitions
# --------------------------------------------------------------------------
def window_pixels(frame: np.ndarray, g: dict, pol: int) -> np.ndarray:
    """The FFT window of `pol` cut from the frame, [Ny][Nx], FP64."""
    gp = g["pols"][pol]
    return np.asarray(frame, dtype=np.float64)[gp["y0"]:gp["y0"] + g["ny"],
                                               gp["x0"]:gp["x0"] + g["nx"]]


def spectrum_window(frame: np.ndarray, g: dict, pol: int) -> np.ndarray:
    """Pipeline steps 1-2: Fourier window M(u,v) I~(u,v), placed on the
    Wy x Wx IFFT grid at (v mod Wy, u mod Wx). I~ is an explicit DFT with
    the pixel coordinates taken relative to the (sub-pixel) beam centre."""
    gp = g["pols"][pol]
    nx, ny, p = g["nx"], g["ny"], g["p"]
    win = window_pixels(frame, g, pol)
    xj = (np.arange(nx) - nx / 2.0) * p - gp["dx"]
    yj = (np.arange(ny) - ny / 2.0) * p - gp["dy"]
    us, vs, m = gp["us"], gp["vs"], gp["mask"]
    # DFT matrices at the needed bins only (the definition needs I~ where M=1)
    dx_mat = np.exp(-2j * np.pi * np.outer(us, xj) / (nx * p))   # [u][x]
    dy_mat = np.exp(-2j * np.pi * np.outer(vs, yj) / (ny * p))   # [v][y]
    spec = dy_mat @ win @ dx_mat.T                                # [v][u]
    out = np.zeros((g["wy"], g["wx"]), dtype=np.complex128)
    for iv, v in enumerate(vs):
        for iu, u in enumerate(us):
            if m[iv, iu]:
                out[v % g["wy"], u % g["wx"]] = spec[iv, iu]
    return out


def field_from_window(window: np.ndarray, g: dict, pol: int) -> np.ndarray:
    """Pipeline step 2 (the IFFT) and the tilt/defocus removal: E(x'_k, y'_l)
    on the field grid, [Fy][Fx]: in IFFT resolution mode 1 the Fourier-window
    size (x'_k = (k - Wx/2) N p / Wx), in mode 0 the FFT size (x'_k =
    (k - Nx/2) p, the camera pixels of the FFT window). The window is the
    same in both modes: the bins, held on the Wy x Wx grid."""
    gp = g["pols"][pol]
    nx, ny, p, lam = g["nx"], g["ny"], g["p"], g["lam"]
    wx, wy = g["wx"], g["wy"]
    xk = (np.arange(g["fx"]) - g["fx"] / 2.0) * g["px2"]
    yl = (np.arange(g["fy"]) - g["fy"] / 2.0) * g["py2"]
    # every window bin (u, v) is represented by its grid cell (u mod W, v mod W);
    # recover the actual lattice bin to evaluate the inverse transform.
    us, vs, m = gp["us"], gp["vs"], gp["mask"]
    ucol = {}
    for iu, u in enumerate(us):
        if m[:, iu].any():
            ucol[u % wx] = u
    vrow = {}
    for iv, v in enumerate(vs):
        if m[iv, :].any():
            vrow[v % wy] = v
    qu = np.array(sorted(ucol))
    qv = np.array(sorted(vrow))
    ub = np.array([ucol[q] for q in qu], dtype=np.float64)
    vb = np.array([vrow[q] for q in qv], dtype=np.float64)
    sub = window[np.ix_(qv, qu)]                                   # [v][u]
    gx = np.exp(2j * np.pi * np.outer(ub, xk) / (nx * p))         # [u][k]
    gy = np.exp(2j * np.pi * np.outer(yl, vb) / (ny * p))         # [l][v]
    e = gy @ sub @ gx / (nx * ny)                                  # [l][k]
    phi = (2 * np.pi * (gp["ax"] * xk[None, :] / (nx * p) + gp["ay"] * yl[:, None] / (ny * p))
           + np.pi * gp["defocus"] * (xk[None, :] ** 2 + yl[:, None] ** 2) / lam)
    return e * np.exp(1j * phi)


def overlap(field: np.ndarray, g: dict, waist: float, group_count: int) -> np.ndarray:
    """Pipeline step 3: c_mn = sum_{k,l} E u_m(x'_k) u_n(y'_l) p'_x p'_y over
    the field grid, for every HG(m,n) with m+n < groupCount, in mode_list
    order."""
    xk = (np.arange(g["fx"]) - g["fx"] / 2.0) * g["px2"]
    yl = (np.arange(g["fy"]) - g["fy"] / 2.0) * g["py2"]
    ux = hermite_gauss_1d(group_count, xk, waist)   # [m][k]
    uy = hermite_gauss_1d(group_count, yl, waist)   # [n][l]
    cm = uy @ field @ ux.T * (g["px2"] * g["py2"])   # [n][m]
    return np.array([cm[n, m] for (m, n) in mode_list(group_count)], dtype=np.complex128)


def power_normalise(coefs: np.ndarray) -> np.ndarray:
    """Per-frame normalisation over both polarisations jointly: c / sqrt(P),
    P = sum |c|^2 (0 stays 0)."""
    c = np.asarray(coefs, dtype=np.complex128)
    pw = float(np.sum(np.abs(c) ** 2))
    return c / math.sqrt(pw) if pw > 0 else np.zeros_like(c)


def process_frame(frame: np.ndarray, params: dict, g: dict | None = None) -> dict:
    """One frame through the whole path: window, field and coefficients per
    polarisation, plus the power-normalised coefficients."""
    if g is None:
        g = geometry(params)
    wins, fields, coefs = [], [], []
    for pol in range(params["pol_count"]):
        w = spectrum_window(frame, g, pol)
        e = field_from_window(w, g, pol)
        wins.append(w)
        fields.append(e)
        if params["max_mg"] > 0:
            coefs.append(overlap(e, g, params["waist"], params["max_mg"]))
        else:
            coefs.append(np.zeros(0, dtype=np.complex128))
    c = np.stack(coefs)
    return dict(window=np.stack(wins), field=np.stack(fields), coefs=c,
                coefs_norm=power_normalise(c.reshape(-1)).reshape(c.shape))


def captured_power(frame: np.ndarray, params: dict, g: dict | None = None):
    """Alignment goal terms ("Automatic (AutoAlign)": the batch insertion loss,
    read as the share of the field's power the HG basis holds): per pol the
    mode power sum |c|^2 and the field power sum |E|^2 p'_x p'_y. Returns two
    arrays [pol]."""
    if g is None:
        g = geometry(params)
    mp, fp = [], []
    for pol in range(params["pol_count"]):
        w = spectrum_window(frame, g, pol)
        e = field_from_window(w, g, pol)
        c = overlap(e, g, params["waist"], params["max_mg"])
        mp.append(float(np.sum(np.abs(c) ** 2)))
        fp.append(float(np.sum(np.abs(e) ** 2)) * g["px2"] * g["py2"])
    return np.array(mp), np.array(fp)


def goal_db(frames, params, indices=None) -> float:
    """10 log10(sum over frames and pols of mode power / field power)."""
    g = geometry(params)
    idx = range(frames.shape[0]) if indices is None else indices
    m = f = 0.0
    for i in idx:
        a, b = captured_power(np.asarray(frames[i], dtype=np.float64), params, g)
        m += a.sum()
        f += b.sum()
    return 10.0 * math.log10(m / f)


def process_batch(frames: np.ndarray, params: dict, indices=None) -> dict:
    """process_frame over frames[i] for i in `indices` (all by default)."""
    g = geometry(params)
    idx = range(frames.shape[0]) if indices is None else indices
    res = [process_frame(frames[i], params, g) for i in idx]
    return {k: np.stack([r[k] for r in res]) for k in res[0]}


# --------------------------------------------------------------------------
# field export in the paper's 16-bit format ("Return reconstructed fields":
# int16 real and imaginary parts and one float scale per field, the field
# being (re + i im) / scale)
# --------------------------------------------------------------------------
INT16_FULL = 32767


def fields_to_int16(field: np.ndarray):
    """One field (complex64 values, any shape) -> (re, im, scale). Reading:
    the scale maps the largest real or imaginary magnitude of the field to
    32767, scale = 32767 / max(|Re|, |Im|) (1 for an all-zero field), and
    each part is rounded to the nearest integer, ties to even. Done in FP32,
    the precision the fields are kept in."""
    f = np.asarray(field, dtype=np.complex64)
    re = f.real.astype(np.float32)
    im = f.imag.astype(np.float32)
    peak = np.float32(max(float(np.abs(re).max(initial=0.0)), float(np.abs(im).max(initial=0.0))))
    scale = np.float32(1.0) if peak == 0 else np.float32(INT16_FULL) / peak
    qr = np.rint(re * scale).astype(np.int16)
    qi = np.rint(im * scale).astype(np.int16)
    return qr, qi, scale
