"""Plain FP64 oracle of the largest Fourier window for a reference tilt.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's background section ("How do you choose the angle of the Reference
Field?") and its AutoAlignFourierWindowRadius option: the window of radius w
around the cross term at tilt t must not meet the autocorrelation terms at the
origin, whose radius is 2w (so |t| >= 3w), nor the conjugate cross term at
-t (radius w, so |2t| >= 2w); without wrapping it must also stay inside the
resolvable spectrum |t_x| + w <= w_max, |t_y| + w <= w_max, and with wrapping
the spectrum is periodic with period 2 w_max along each axis, so the same
separations hold from every periodic image instead. Everything is in angles
(degrees), where the window is a circle. With two polarisations the window
radius is one, so the smaller of the two pols' largest radii is taken.
"""
from __future__ import annotations

import math


def max_window_radius(tilts_deg, w_max_deg: float, wrap: bool = False) -> float:
    """Largest window radius (degrees) for every tilt (tx, ty) in `tilts_deg`."""
    best = math.inf
    for tx, ty in tilts_deg:
        if not wrap:
            w = min(math.hypot(tx, ty) / 3.0, w_max_deg - abs(tx), w_max_deg - abs(ty))
        else:
            w = math.inf
            period = 2.0 * w_max_deg
            for kx in range(-2, 3):
                for ky in range(-2, 3):
                    # the autocorrelation terms at the image (kx, ky) of the origin
                    w = min(w, math.hypot(tx - kx * period, ty - ky * period) / 3.0)
                    # the conjugate cross term at the image of -t: |t - (-t + k P)| >= 2 w
                    w = min(w, math.hypot(2 * tx - kx * period, 2 * ty - ky * period) / 2.0)
        best = min(best, w)
    return max(best, 0.0)
