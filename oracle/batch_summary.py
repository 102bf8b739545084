"""FP64 oracle of the batch summary (Advanced functions: digHoloBatchGetSummary;
"Analysis parameter types").

TEST INFRASTRUCTURE ONLY (see the package docstring).

For every batch element and polarisation, the paper analyses two planes: the
Fourier plane of the camera (the result of the FFT) and the reconstructed
field plane (the result of the IFFT after tilt removal), and it does the same
for the whole batch. Seven parameters are named: total power, centre of mass
along x and y, the largest absolute value and its index, the effective area
(Petermann II) and the centre of mass along y with the y axis taken as
periodic. The paper gives no formulas; the readings taken here:

* intensity I = |z|^2 of the plane's complex values; dA = |dx dy|, the cell of
  the plane's axes;
* TOTALPOWER = sum I dA;  COMX = sum x I / sum I;  COMY likewise;
* MAXABS = max |z| = sqrt(max I); MAXABSIDX = the row-major index l W + k of
  the first pixel (lowest index) holding it;
* AEFF = (sum I dA)^2 / (sum I^2 dA), so that a Gaussian beam with
  I ~ exp(-2 r^2 / w^2) has AEFF = pi w^2;
* COMYWRAP: the circular mean of y over the period L = H dy of the axis,
  y_0 + L arg(sum I exp(2 pi i (y - y_0) / L)) / (2 pi), the angle taken in
  [0, 2 pi) so the result lies in the axis' range;
* an all-zero plane gives zeros (index 0);
* the batch entry (the paper's "+1") is the same analysis of the intensity
  summed over the batch (the paper's totalIntensity);
* Fourier plane: the real-to-complex half plane of each polarisation's FFT
  window, kx = 0 .. Nx/2 (width Nx/2 + 1) by ky = -Ny/2 .. Ny/2 - 1 (height
  Ny, ascending), with the axes in degrees of paraxial angle (bin k at
  k lambda / (N p) radians), the units of the reference tilt;
* field plane: the reconstructed field on its grid (x'_k = (k - W/2) p' in
  metres from the beam centre).
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import DEG, geometry, window_pixels

PARAMETERS = ("TOTALPOWER", "COMX", "COMY", "MAXABS", "MAXABSIDX", "AEFF", "COMYWRAP")


def plane_parameters(intensity: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """The seven parameters of one plane of intensity [H][W] on axes x [W], y [H]."""
    i = np.asarray(intensity, dtype=np.float64)
    h, w = i.shape
    dx = abs(x[1] - x[0]) if w > 1 else 1.0
    dy = abs(y[1] - y[0]) if h > 1 else 1.0
    da = dx * dy
    s = float(i.sum())
    out = np.zeros(len(PARAMETERS))
    if not s > 0.0:
        return out
    flat = i.ravel()
    k = int(np.argmax(flat))                       # first occurrence of the maximum
    out[0] = s * da
    out[1] = float(i.sum(axis=0) @ x) / s
    out[2] = float(i.sum(axis=1) @ y) / s
    out[3] = math.sqrt(flat[k])
    out[4] = k
    out[5] = (s * da) ** 2 / (float((i * i).sum()) * da)
    period = h * dy
    z = complex(i.sum(axis=1) @ np.exp(2j * math.pi * (y - y[0]) / period))
    ang = math.atan2(z.imag, z.real) % (2.0 * math.pi)
    out[6] = y[0] + period * ang / (2.0 * math.pi)
    return out


def fourier_axes(params: dict):
    """Axes (degrees) of the half Fourier plane of a pol window."""
    g = geometry(params)
    nx, ny, p, lam = g["nx"], g["ny"], params["pixel_size"], params["wavelength"]
    x = np.arange(nx // 2 + 1) * lam / (nx * p) / DEG
    y = (np.arange(ny) - ny // 2) * lam / (ny * p) / DEG
    return x, y


def fourier_plane(frame: np.ndarray, params: dict, pol: int) -> np.ndarray:
    """|FFT|^2 of the pol's window on the half plane [Ny][Nx/2+1] by explicit
    DFT matrices (rows: ky ascending from -Ny/2)."""
    g = geometry(params)
    nx, ny = g["nx"], g["ny"]
    win = window_pixels(frame, g, pol)
    kx = np.arange(nx // 2 + 1)
    ky = np.arange(ny) - ny // 2
    dxm = np.exp(-2j * math.pi * np.outer(kx, np.arange(nx)) / nx)      # [kx][x]
    dym = np.exp(-2j * math.pi * np.outer(ky, np.arange(ny)) / ny)      # [ky][y]
    f = dym @ win @ dxm.T
    return f.real ** 2 + f.imag ** 2


def field_axes(params: dict):
    """Axes (metres from the beam centre) of the reconstructed field, on the
    IFFT grid (IFFT resolution mode 1) or the FFT grid (mode 0)."""
    g = geometry(params)
    x = (np.arange(g["fx"]) - g["fx"] / 2.0) * g["px2"]
    y = (np.arange(g["fy"]) - g["fy"] / 2.0) * g["py2"]
    return x, y


def summarise(intensities: np.ndarray, x: np.ndarray, y: np.ndarray):
    """intensities [B][P][H][W] -> (parameters [7][P][B+1], summed intensity [P][H][W])."""
    b, npol = intensities.shape[:2]
    out = np.zeros((len(PARAMETERS), npol, b + 1))
    total = intensities.sum(axis=0)
    for p in range(npol):
        for e in range(b):
            out[:, p, e] = plane_parameters(intensities[e, p], x, y)
        out[:, p, b] = plane_parameters(total[p], x, y)
    return out, total


def batch_summary_fourier(frames: np.ndarray, params: dict):
    """Plane 0 of a batch of frames: (parameters, summed intensity, x, y)."""
    x, y = fourier_axes(params)
    inten = np.stack([np.stack([fourier_plane(f, params, p) for p in range(params["pol_count"])]) for f in frames])
    par, total = summarise(inten, x, y)
    return par, total, x, y


def batch_summary_field(fields: np.ndarray, params: dict):
    """Plane 1 of a batch of fields [B][P][Wy][Wx]: (parameters, summed intensity, x, y)."""
    x, y = field_axes(params)
    f = np.asarray(fields, dtype=np.complex128)
    par, total = summarise(f.real ** 2 + f.imag ** 2, x, y)
    return par, total, x, y
