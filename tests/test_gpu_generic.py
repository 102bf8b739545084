"""Window sizes without a compiled transform ("Window sizes": the FFT window
is any multiple of 16, the Fourier window radius is free): the runtime-length
row, column and export kernels through the C ABI, against the FP64 oracle
(rel-L2 <= 1e-5 per frame and pol on the window, coefficients and fields)."""
import math

import numpy as np
import pytest

import dh_synth
from tests.test_gpu_parity import _say, check_frames, run_gpu

pytestmark = pytest.mark.gpu

WMAX_DEG = math.degrees(1565e-9 / (2 * 20e-6))


def _cfg(frame_w, frame_h, pols, fft_w, fft_h, radius, groups, waist, dtype="f32", **extra):
    """The 640x512 recipe's noise and seeds on another geometry."""
    cfg = dh_synth.config(1)
    p = dict(cfg["params"], frame_w=frame_w, frame_h=frame_h, pol_count=pols, fft_w=fft_w, fft_h=fft_h,
             window_radius_deg=radius * WMAX_DEG, max_mg=groups, waist=waist, input_dtype=dtype, **extra)
    return dict(cfg, params=p, truth=dict(p), dtype=dtype)


CASES = {
    # id: (geometry, expected generic flags: bit 0 row pass, bit 1 column pass)
    "384x256_r025": (dict(frame_w=384, frame_h=256, pols=1, fft_w=384, fft_h=256, radius=0.25, groups=9,
                          waist=400e-6), 3),
    "2pol_272x304": (dict(frame_w=544, frame_h=304, pols=2, fft_w=272, fft_h=304, radius=0.32, groups=5,
                          waist=300e-6), 3),
    "u16_480": (dict(frame_w=480, frame_h=480, pols=1, fft_w=480, fft_h=480, radius=0.3, groups=12, waist=400e-6,
                     dtype="u16"), 3),
    "1008x512": (dict(frame_w=1008, frame_h=512, pols=1, fft_w=1008, fft_h=512, radius=0.28, groups=6,
                      waist=400e-6), 3),
    "2032x64_prime127": (dict(frame_w=2032, frame_h=64, pols=1, fft_w=2032, fft_h=64, radius=0.32, groups=3,
                              waist=150e-6), 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_generic_sizes_vs_oracle(name):
    geo, flags = CASES[name]
    cfg = _cfg(**geo)
    f, _ = dh_synth.make_frames(cfg, n_frames=3)
    p = cfg["params"]
    _say(f"generic sizes {name}: window {p['fft_w']}x{p['fft_h']}, {f.shape[0]} frames")
    gpu = run_gpu(p, f, keep=True, path="spectral")
    assert gpu["info"].generic == flags, gpu["info"].generic
    check_frames(p, f, gpu, range(f.shape[0]))


@pytest.mark.parametrize("name", ["384x256_r025", "2pol_272x304"])
def test_generic_sizes_mode0_fields(name):
    """IFFT mode 0 on generic lengths: coefficients and the full-size fields
    (the generic export kernels)."""
    cfg = _cfg(**CASES[name][0])
    f, _ = dh_synth.make_frames(cfg, n_frames=2)
    p = dict(cfg["params"], ifft_mode=0)
    _say(f"generic sizes {name}, IFFT mode 0 with fields")
    gpu = run_gpu(p, f, keep=True)
    assert gpu["field"].shape[2:] == (p["fft_h"], p["fft_w"])
    check_frames(p, f, gpu, range(2))


def test_generic_sizes_batch_bit_identical_alone():
    """A frame's coefficients do not depend on its batch on the generic
    kernels either (fixed reduction order)."""
    cfg = _cfg(**CASES["384x256_r025"][0])
    f, _ = dh_synth.make_frames(cfg, n_frames=5)
    p = cfg["params"]
    batch = run_gpu(p, f, keep=False, path="spectral")
    alone = run_gpu(p, f[3:4], keep=False, path="spectral")
    assert np.array_equal(batch["coefs"][3], alone["coefs"][0])
