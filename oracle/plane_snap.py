"""Plain FP64 oracle of the AutoAlign snap's first guess of the tilt, made
from the whole Fourier plane.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's "AutoAlign operation modes" section: the snap discards the
current alignment and makes a best guess of where the off-axis term lies in
Fourier space; it is reliable for the tilt. No formula is given. Readings
taken here:

  * the power spectrum |FFT|^2 of each polarisation's FFT window, summed over
    the first n frames (32);
  * the zero-order terms (|R|^2 at the origin and |S|^2 about it, whose
    radius is twice the window's) are left out: every bin inside the ellipse
    of twice the window radius about the origin;
  * the brightest bin left, b, and its mirror -b are the two cross terms (the
    frame is real, so both carry the same power). The term sitting at bin c
    has tilt -c (the SR* term sits at minus the tilt); of the two, the one
    whose tilt lies nearer the starting tilt (in degrees) is taken, and from
    an equidistant start (a zero tilt) the one with positive x tilt, then
    positive y;
  * its position is the power-weighted centroid, with weights the power above
    the mean of the bins left in, over the window-radius ellipse about its
    brightest bin; the bin offsets are taken periodically (a term may
    straddle the edge of the plane). The tilt is minus that position.
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import geometry

SNAP_FRAMES = 32


def plane_power(frames: np.ndarray, params: dict, n_frames: int = SNAP_FRAMES) -> np.ndarray:
    """[pol][u][v]: |FFT|^2 of each pol's FFT window summed over the first
    n_frames frames (u, v the bin indices 0 .. N-1 along x and y)."""
    g = geometry(params)
    n = min(n_frames, frames.shape[0])
    out = np.zeros((params["pol_count"], g["nx"], g["ny"]))
    for b in range(n):
        f = np.asarray(frames[b], dtype=np.float64)
        for pol in range(params["pol_count"]):
            gp = g["pols"][pol]
            w = f[gp["y0"]:gp["y0"] + g["ny"], gp["x0"]:gp["x0"] + g["nx"]]   # [y][x]
            out[pol] += (np.abs(np.fft.fft2(w)) ** 2).T
    return out


def _signed(k: int, n: int) -> int:
    return k if k < n // 2 else k - n


def snap_tilt_plane(frames: np.ndarray, params: dict, n_frames: int = SNAP_FRAMES):
    """The snap's tilt per pol ([pol][x, y], degrees) from the whole Fourier
    plane, with params' tilt as the starting tilt."""
    g = geometry(params)
    nx, ny, rx, ry = g["nx"], g["ny"], g["rx"], g["ry"]
    binx = params["wavelength"] / (nx * params["pixel_size"]) / (math.pi / 180.0)   # degrees per bin
    biny = params["wavelength"] / (ny * params["pixel_size"]) / (math.pi / 180.0)
    power = plane_power(frames, params, n_frames)
    us = np.array([_signed(k, nx) for k in range(nx)], dtype=np.float64)
    vs = np.array([_signed(k, ny) for k in range(ny)], dtype=np.float64)
    zero = (us[:, None] / (2.0 * rx)) ** 2 + (vs[None, :] / (2.0 * ry)) ** 2 <= 1.0
    tilts = []
    for pol in range(params["pol_count"]):
        pw = power[pol]
        mean = float(pw[~zero].mean())
        j, i = np.unravel_index(int(np.argmax(np.where(zero, -np.inf, pw))), pw.shape)
        bu, bv = int(us[j]), int(vs[i])
        t0x, t0y = params["tilt_deg"][pol]
        d1 = math.hypot(-bu * binx - t0x, -bv * biny - t0y)     # the term at b: tilt -b
        d2 = math.hypot(bu * binx - t0x, bv * biny - t0y)       # its mirror at -b: tilt b
        first = d1 < d2 if d1 != d2 else (-bu > 0 or (-bu == 0 and -bv > 0))
        cu, cv = (bu, bv) if first else (-bu, -bv)
        sw = su = sv = 0.0
        for du in range(-math.ceil(rx), math.ceil(rx) + 1):
            for dv in range(-math.ceil(ry), math.ceil(ry) + 1):
                if (du / rx) ** 2 + (dv / ry) ** 2 > 1.0:
                    continue
                w = max(0.0, float(pw[(cu + du) % nx, (cv + dv) % ny]) - mean)
                sw += w
                su += w * du
                sv += w * dv
        uc = cu + (su / sw if sw > 0 else 0.0)
        vc = cv + (sv / sw if sw > 0 else 0.0)
        tilts.append([-uc * binx, -vc * biny])
    return tilts
