"""Plain FP64 oracle of the AutoAlign snap estimates of beam centre and waist.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's AutoAlign section says that the snap stage makes a first guess of
the tilt, the beam centre and, when the number of mode groups is right, the
waist, and that it is reliable for tilt and beam centre and only moderately
so for the waist. It gives no formula. The readings taken here:

  beam centre  the centroid of the batch's reconstructed intensity |E|^2 on
               the coarse grid x'_k = (k - Wx/2) p'_x, which is centred on the
               current beam centre: c_new = c + sum x'|E|^2 / sum |E|^2 (and y).
  waist        the pooled central second moment of |E|^2 over the batch and
               both polarisations, read with the assumption that the power is
               spread evenly over the HG modes of G groups. For HG_mn,
               <x^2> = w^2 (2m + 1) / 4 (w the 1/e^2 intensity radius); over
               the modes m + n < G the mean of m is (G - 1) / 3, so
               <x^2> = <y^2> = w^2 (2G + 1) / 12 and
               w = sqrt(6 (<x^2> + <y^2>) / (2G + 1)).
  defocus      the paper says the snap finds its magnitude only. A defocus D
               is the phase pi D r^2 / lambda on the field, whose gradient
               2 pi D r / lambda widens the angular spectrum:
               <kx^2> + <ky^2> = K_S + a^2 (<x^2> + <y^2>), a = 2 pi D / lambda,
               with K_S the angular spread of the modes themselves; for HG_mn
               <kx^2> = (2m + 1) / w^2, so with the power spread evenly over G
               groups K_S = 2 (2G + 1) / (3 w^2). Per pol, <k^2> is the central
               second moment of the batch's window power |M I~|^2 over the
               window bins (k = 2 pi u / (N p)) and <x^2> + <y^2> the central
               second moment of |E|^2; |D| = lambda a / (2 pi) with
               a^2 = max(0, (<k^2> - K_S) / (<x^2> + <y^2>)).
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import field_from_window, geometry, spectrum_window, window_pixels


def field_moments(field: np.ndarray, g: dict) -> np.ndarray:
    """[sum I, sum x' I, sum y' I, sum x'^2 I, sum y'^2 I] of I = |E|^2 over
    the field grid of one field [Fy][Fx] (coordinates relative to the beam
    centre, in metres)."""
    fx, fy = g["fx"], g["fy"]
    xk = (np.arange(fx) - fx / 2.0) * g["px2"]
    yl = (np.arange(fy) - fy / 2.0) * g["py2"]
    i = np.abs(np.asarray(field, dtype=np.complex128)) ** 2
    ix = i.sum(axis=0)          # over y: a function of x
    iy = i.sum(axis=1)          # over x: a function of y
    return np.array([i.sum(), (xk * ix).sum(), (yl * iy).sum(), (xk * xk * ix).sum(), (yl * yl * iy).sum()])


def batch_moments(frames: np.ndarray, params: dict, indices=None) -> np.ndarray:
    """field_moments summed over the frames, per polarisation: [pol][5]."""
    g = geometry(params)
    idx = range(frames.shape[0]) if indices is None else indices
    out = np.zeros((params["pol_count"], 5))
    for b in idx:
        f = np.asarray(frames[b], dtype=np.float64)
        for pol in range(params["pol_count"]):
            out[pol] += field_moments(field_from_window(spectrum_window(f, g, pol), g, pol), g)
    return out


def snap_centre_waist(frames: np.ndarray, params: dict, indices=None):
    """The snap's beam centre per pol ([pol][x, y], metres) and waist (metres)
    from the batch's reconstructed fields at `params`."""
    mom = batch_moments(frames, params, indices)
    centre = []
    mxx = myy = total = 0.0
    for pol in range(params["pol_count"]):
        s, sx, sy, sxx, syy = mom[pol]
        cx, cy = params["beam_centre"][pol]
        centre.append([cx + sx / s, cy + sy / s])
        mxx += sxx - sx * sx / s
        myy += syy - sy * sy / s
        total += s
    g = params["max_mg"]
    waist = math.sqrt(6.0 * (mxx + myy) / total / (2 * g + 1))
    return centre, waist


def snap_defocus_magnitude(frames: np.ndarray, params: dict, waist: float, indices=None):
    """The snap's defocus magnitude per pol (dioptre) from the batch at params
    (its tilt the snapped one), with `waist` in K_S."""
    g = geometry(params)
    mom = batch_moments(frames, params, indices)
    idx = range(frames.shape[0]) if indices is None else indices
    nx, ny, p, lam = g["nx"], g["ny"], g["p"], g["lam"]
    kx, ky = 2.0 * math.pi / (nx * p), 2.0 * math.pi / (ny * p)
    ks = 2.0 * (2 * params["max_mg"] + 1) / (3.0 * waist * waist)
    out = []
    for pol in range(params["pol_count"]):
        gp = g["pols"][pol]
        us, vs, m = gp["us"], gp["vs"], gp["mask"]
        xj = np.arange(nx) * p
        yj = np.arange(ny) * p
        dx_mat = np.exp(-2j * np.pi * np.outer(us, xj) / (nx * p))
        dy_mat = np.exp(-2j * np.pi * np.outer(vs, yj) / (ny * p))
        pw = np.zeros((len(vs), len(us)))
        for b in idx:
            win = window_pixels(np.asarray(frames[b], dtype=np.float64), g, pol)
            pw += np.abs(dy_mat @ win @ dx_mat.T) ** 2
        pw = np.where(m, pw, 0.0)
        w0 = pw.sum()
        uu, vv = np.asarray(us, dtype=np.float64)[None, :], np.asarray(vs, dtype=np.float64)[:, None]
        mu, mv = (pw * uu).sum() / w0, (pw * vv).sum() / w0
        k2 = kx * kx * (pw * (uu - mu) ** 2).sum() / w0 + ky * ky * (pw * (vv - mv) ** 2).sum() / w0
        s, sx, sy, sxx, syy = mom[pol]
        spread = (sxx - sx * sx / s) / s + (syy - sy * sy / s) / s
        out.append(math.sqrt(max(0.0, (k2 - ks) / spread)) * lam / (2.0 * math.pi))
    return out
