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
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import field_from_window, geometry, spectrum_window


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
