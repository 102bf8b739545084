"""Plain FP64 oracle of wavelength sweeps and frame averaging.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's "Wavelength" and "Input/output wavelength ordering" sections: a
batch can hold frames taken at L wavelengths; the wavelength is the fast axis
of the frames (adjacent frames differ in wavelength) or the slow one (all
frames of one wavelength together), for the input frames and, separately,
for the output fields and coefficients. Its "SetBatchAvg" and "Averaging
modes" sections: A frames are averaged into one output; their Fourier windows
are added in phase (a phase shift per frame compensates the reference beam's
drift) and one IFFT follows; the frames of an output are adjacent
(sequential, AAABBB), a whole batch apart (interlaced, ABCABC), or whole
wavelength sweeps apart (sequential sweep, {A}{A}{B}{B}, the same as
sequential for one wavelength). Readings taken here:

  * N outputs = I inputs x L wavelengths; output o holds input i at
    wavelength w: o = i L + w (fast) or w I + i (slow). N must be a multiple
    of L.
  * without averaging, frame j of the batch holds (i, w) by the input
    ordering, j = i L + w (fast) or w I + i (slow); with averaging the
    repetition a of (i, w) is frame j A + a (sequential), a N + j
    (interlaced) or (i A + a) L + w (sequential sweep: a sweep is L adjacent
    frames, whatever the input ordering).
  * each frame is processed at its own wavelength: the tilt angle and the
    defocus are converted with that wavelength, while the window radius in
    bins, the IFFT size and the field grid are those of the plan's centre
    wavelength (the params' "wavelength"), so every output has one shape.
  * the phase of repetition a is arg sum W_a conj(W_0) over both
    polarisations and every window bin (W_0: the first repetition), and the
    output window is the mean of W_a exp(-i phase_a); the field and the
    coefficients follow from that window as for a single frame.
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import field_from_window, geometry, mask_bins, overlap, power_normalise, spectrum_window

SEQUENTIAL, INTERLACED, SEQUENTIAL_SWEEP = 0, 1, 2
FAST, SLOW = 0, 1


def frame_index_map(n_out: int, avg_count: int, avg_mode: int, wl_count: int, in_order: int, out_order: int):
    """(wavelength index of every output, input frame indices of every
    output's repetitions [n_out][avg_count])."""
    if n_out % wl_count:
        raise ValueError("the outputs are not a whole number of sweeps")
    n_in = n_out // wl_count
    lam = np.zeros(n_out, dtype=np.int64)
    frames = np.zeros((n_out, avg_count), dtype=np.int64)
    for i in range(n_in):
        for w in range(wl_count):
            o = i * wl_count + w if out_order == FAST else w * n_in + i
            j = i * wl_count + w if in_order == FAST else w * n_in + i
            lam[o] = w
            for a in range(avg_count):
                if avg_mode == SEQUENTIAL:
                    frames[o, a] = j * avg_count + a
                elif avg_mode == INTERLACED:
                    frames[o, a] = a * n_out + j
                else:
                    frames[o, a] = (i * avg_count + a) * wl_count + w
    return lam, frames


def at_wavelength(params: dict, lam: float) -> dict:
    """Geometry of one wavelength of a sweep: window radius, IFFT size and
    field grid of the centre wavelength; tilt bins, mask position and phases
    of `lam`."""
    g0 = geometry(params)
    g = geometry(dict(params, wavelength=lam))
    for k in ("rx", "ry", "wx", "wy", "px2", "py2", "fx", "fy"):
        g[k] = g0[k]
    pols = []
    for gp in g["pols"]:
        ax, ay = gp["ax"], gp["ay"]
        us = np.arange(int(math.floor(-ax - g["rx"])) - 1, int(math.ceil(-ax + g["rx"])) + 2)
        vs = np.arange(int(math.floor(-ay - g["ry"])) - 1, int(math.ceil(-ay + g["ry"])) + 2)
        pols.append(dict(gp, us=us, vs=vs, mask=mask_bins(ax, ay, g["rx"], g["ry"], us, vs)))
    g["pols"] = pols
    return g


def average_windows(windows: np.ndarray):
    """windows [A][pol][Wy][Wx] of one output -> (the phase-aligned mean, the
    phases)."""
    w = np.asarray(windows, dtype=np.complex128)
    ph = np.zeros(w.shape[0])
    acc = np.zeros_like(w[0])
    for a in range(w.shape[0]):
        dot = np.sum(w[a] * np.conj(w[0]))
        ph[a] = 0.0 if (a == 0 or dot == 0) else float(np.angle(dot))
        acc += w[a] * np.exp(-1j * ph[a])
    return acc / w.shape[0], ph


def process_sweep(frames: np.ndarray, params: dict, wavelengths, avg_count: int = 1, avg_mode: int = SEQUENTIAL,
                  in_order: int = FAST, out_order: int = FAST, n_out: int | None = None, outputs=None) -> dict:
    """Outputs `outputs` (all by default) of a batch of n_out outputs: window,
    field, coefficients (raw and normalised) per output, [len][pol][...]."""
    lams = list(wavelengths)
    if n_out is None:
        n_out = frames.shape[0] // avg_count
    lam_idx, idx = frame_index_map(n_out, avg_count, avg_mode, len(lams), in_order, out_order)
    geos = [at_wavelength(params, lam) for lam in lams]
    sel = range(n_out) if outputs is None else outputs
    out = {"window": [], "field": [], "coefs": [], "coefs_norm": [], "phase": []}
    for o in sel:
        g = geos[lam_idx[o]]
        wins = np.stack([np.stack([spectrum_window(np.asarray(frames[j], dtype=np.float64), g, pol)
                                   for pol in range(params["pol_count"])]) for j in idx[o]])
        win, ph = average_windows(wins)
        fields = [field_from_window(win[pol], g, pol) for pol in range(params["pol_count"])]
        if params["max_mg"] > 0:
            c = np.stack([overlap(fields[pol], g, params["waist"], params["max_mg"])
                          for pol in range(params["pol_count"])])
        else:
            c = np.zeros((params["pol_count"], 0), dtype=np.complex128)
        out["window"].append(win)
        out["field"].append(np.stack(fields))
        out["coefs"].append(c)
        out["coefs_norm"].append(power_normalise(c.reshape(-1)).reshape(c.shape))
        out["phase"].append(ph)
    return {k: np.stack(v) for k, v in out.items()}
