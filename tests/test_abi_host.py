"""Host-only checks of the C ABI: the library loads, exports what
include/dh.h declares, validates parameters with the paper's error codes and
derives the same geometry as the oracle. No GPU work is launched."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import dh_synth
import oracle
import paper_2204_02348_amd as dh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dh.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(dh_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "dh_plan" in names and "dh_process_batch" in names and "dh_mode_coefs" in names
    L = ctypes.CDLL(dh.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(dh.EXPORTS) == names


def _p(idx=1, **kw):
    d = dict(dh_synth.config(idx)["params"])
    d.update(kw)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(pol_count=3), dh.ERR_INVALIDPOLARISATION),
    (dict(pol_count=0), dh.ERR_INVALIDPOLARISATION),
    (dict(frame_w=650), dh.ERR_INVALIDDIMENSION),
    (dict(frame_h=0), dh.ERR_INVALIDDIMENSION),
    (dict(fft_w=8), dh.ERR_INVALIDDIMENSION),
    (dict(fft_w=336), dh.ERR_INVALIDDIMENSION),          # window 0 would leave the frame
    (dict(pixel_size=0.0), dh.ERR_INVALIDARGUMENT),
    (dict(wavelength=-1.0), dh.ERR_INVALIDARGUMENT),
    (dict(window_radius_deg=0.0), dh.ERR_INVALIDARGUMENT),
    (dict(window_radius_deg=5.0), dh.ERR_INVALIDARGUMENT),  # wider than the spectrum
    (dict(waist=0.0), dh.ERR_INVALIDARGUMENT),
    (dict(max_mg=-1), dh.ERR_INVALIDARGUMENT),
    (dict(max_mg=101), dh.ERR_INVALIDARGUMENT),          # past the paper's 100 LG groups
    (dict(max_mg=33, path="field"), dh.ERR_INVALIDARGUMENT),    # the field path's overlap: G <= 32
    (dict(max_mg=40, keep_fields=1), dh.ERR_INVALIDARGUMENT),   # mode-1 fields need the field path
    (dict(max_mg=64, precision="split_fp16"), dh.ERR_INVALIDARGUMENT),
    (dict(input_dtype=7), dh.ERR_INVALIDARGUMENT),
    (dict(precision=9), dh.ERR_INVALIDARGUMENT),
    (dict(ifft_mode=2), dh.ERR_INVALIDARGUMENT),
    (dict(ifft_mode=0, path="field"), dh.ERR_INVALIDARGUMENT),        # mode 0 runs the spectral path
    (dict(ifft_mode=0, precision="split_bf16"), dh.ERR_INVALIDARGUMENT),
    (dict(ifft_mode=0, max_mg=0, path="field"), dh.ERR_INVALIDARGUMENT),
    (dict(path=3), dh.ERR_INVALIDARGUMENT),
    (dict(path=-1), dh.ERR_INVALIDARGUMENT),
    (dict(path="spectral", keep_fields=1), dh.ERR_INVALIDARGUMENT),
    (dict(path="spectral", precision="split_bf16"), dh.ERR_INVALIDARGUMENT),
    (dict(path="spectral", max_mg=0), dh.ERR_INVALIDARGUMENT),
    (dict(beam_centre=[[400 * 20e-6, 0], [0, 0]]), dh.ERR_INVALIDDIMENSION),
])
def test_validation_error_codes(kw, code):
    rc, _ = dh.plan_check(_p(**kw))
    assert rc == code


@pytest.mark.parametrize("kw", [dict(max_mg=33), dict(max_mg=64), dict(max_mg=100),
                                dict(max_mg=100, ifft_mode=0, keep_fields=1)])
def test_large_group_counts_take_the_spectral_path(kw):
    # G above 32 runs the spectral contraction in chunks of 32 mode columns;
    # IFFT mode 0 exports its fields from the kept window
    d = _p(3, **kw)
    d.update(dh_synth.config(3, 3)["params"], **kw)
    rc, info = dh.plan_check(d)
    assert rc == 0 and info.path == dh.PATH_SPECTRAL
    assert info.modes == kw["max_mg"] * (kw["max_mg"] + 1) // 2


def test_mode0_without_decomposition():
    # IFFT mode 0 with G = 0: the field reconstruction alone (the paper's
    # field-reconstruction benchmarks run without a decomposition)
    rc, info = dh.plan_check(_p(1, ifft_mode=0, max_mg=0, keep_fields=1))
    assert rc == 0 and info.path == dh.PATH_SPECTRAL and info.modes == 0
    assert (info.field_w, info.field_h) == (320, 512)


COMPILED = (64, 128, 256, 320, 512, 640, 1024, 2048)      # transform lengths with compiled kernels


def test_every_window_size_multiple_of_16():
    # "Window sizes": any multiple of 16 from 64 to 2048 along either axis
    # (compiled transforms or the runtime-length kernels), on the spectral path
    base = dict(dh_synth.config(3, 1)["params"], input_dtype="f32")
    for n in range(64, 2049, 16):
        for fw, fh in ((n, n), (n, 256), (384, n)):
            rc, info = dh.plan_check(dict(base, frame_w=fw, frame_h=fh, fft_w=fw, fft_h=fh))
            assert rc == 0 and info.path == dh.PATH_SPECTRAL, (fw, fh, rc)
            # bit 0: the row pass runs the runtime-length kernel exactly when N_x has no compiled one
            assert bool(info.generic & 1) == (fw not in COMPILED), (fw, fh, info.generic)
            if fh not in COMPILED:
                assert info.generic & 2, (fw, fh)


def test_generic_sizes_keep_the_field_path_out():
    # the field path (mode-1 fields, split precision, AutoAlign trials) needs
    # compiled transforms for every length
    d = dict(dh_synth.config(3, 1)["params"], input_dtype="f32", frame_w=384, frame_h=256, fft_w=384, fft_h=256)
    assert dh.plan_check(d)[0] == 0
    assert dh.plan_check(dict(d, keep_fields=1))[0] == dh.ERR_INVALIDDIMENSION
    assert dh.plan_check(dict(d, precision="split_bf16"))[0] == dh.ERR_INVALIDDIMENSION
    assert dh.plan_check(dict(d, ifft_mode=0, keep_fields=1))[0] == 0


def test_null_pointer():
    assert dh.lib().dh_plan_check(None, 1, None) == dh.ERR_NULLPOINTER
    h = ctypes.c_int()
    assert dh.lib().dh_plan(None, 1, 0, ctypes.byref(h)) == dh.ERR_NULLPOINTER


def test_invalid_handles_without_gpu():
    L = dh.lib()
    assert L.dh_destroy(12345) == dh.ERR_INVALIDHANDLE
    assert L.dh_last_error(-1) == dh.ERR_INVALIDHANDLE
    b = ctypes.c_int(7)
    m = ctypes.c_int(7)
    assert L.dh_mode_coefs(999, None, None, ctypes.byref(b), ctypes.byref(m), None, 1) == dh.ERR_INVALIDHANDLE
    assert b.value == 0 and m.value == 0   # getters zero their outputs on a bad handle
    assert L.dh_set_align_goal(999, 0, 0, 0) == dh.ERR_INVALIDHANDLE
    out = (ctypes.c_double * 9)()
    assert L.dh_transfer_metrics(999, 0, 0, out) == dh.ERR_INVALIDHANDLE


def test_window_size_floored_to_16():
    rc, info = dh.plan_check(_p(0, fft_w=130, fft_h=143))
    assert rc == 0 and info.fft_w == 128 and info.fft_h == 128


@pytest.mark.parametrize("idx,cam", [(0, 0), (1, 0), (2, 0), (3, 0), (3, 1), (3, 2), (3, 3), (4, 0)])
def test_plan_geometry_matches_oracle(idx, cam):
    cfg = dh_synth.config(idx, cam)
    d = cfg["truth"]
    rc, info = dh.plan_check(d, cfg["frames"])
    assert rc == 0
    g = oracle.geometry(d)
    assert (info.ifft_w, info.ifft_h) == (g["wx"], g["wy"])
    assert info.modes == oracle.mode_count(d["max_mg"])
    assert math.isclose(info.rx, g["rx"], rel_tol=1e-14) and math.isclose(info.ry, g["ry"], rel_tol=1e-14)
    assert math.isclose(info.pitch_x, g["px2"], rel_tol=1e-14)
    bw = 0
    for pol, gp in enumerate(g["pols"]):
        assert (info.x0[pol], info.y0[pol]) == (gp["x0"], gp["y0"])
        assert math.isclose(info.ax[pol], gp["ax"], rel_tol=1e-14)
        cols = gp["us"][gp["mask"].any(axis=0)]
        bw = max(bw, cols.max() - cols.min() + 1)
    # the box is the fixed bound floor(2r)+1 of every window position
    assert info.box_w == math.floor(2 * g["rx"]) + 1 >= bw
    assert info.device_bytes > 0 and info.chunk >= 1


def test_hbm_budget_is_checked_before_allocating():
    # the budget check happens before any device call, so it runs here too
    h = ctypes.c_int(-1)
    p = dh.make_params(_p())
    assert dh.lib().dh_plan(ctypes.byref(p), 1000, 1024, ctypes.byref(h)) == dh.ERR_MEMORYALLOCATION


def test_serving_rejects_bad_arguments_without_gpu():
    L = dh.lib()
    s = ctypes.c_int(-1)
    assert L.dh_serve_create(None, 1, 8, 0, 1, 1, ctypes.byref(s)) == dh.ERR_NULLPOINTER
    hs = (ctypes.c_int * 2)(777, 778)
    assert L.dh_serve_create(hs, 2, 8, 0, 1, 1, ctypes.byref(s)) == dh.ERR_INVALIDHANDLE
    assert L.dh_serve_create(hs, 0, 8, 0, 1, 1, ctypes.byref(s)) == dh.ERR_INVALIDDIMENSION
    assert L.dh_serve_destroy(55) == dh.ERR_INVALIDHANDLE
    assert L.dh_serve_progress(55, None) == dh.ERR_INVALIDHANDLE
    n = ctypes.c_int()
    assert L.dh_serve_submit(55, 0, None, None) == dh.ERR_INVALIDHANDLE


@pytest.mark.parametrize("idx,cam,kw,path", [
    (1, 0, {}, dh.PATH_SPECTRAL),                                  # 640x512 G=9 FP32: spectral
    (1, 0, dict(keep_fields=1), dh.PATH_FIELD),                    # fields requested
    (1, 0, dict(precision="split_bf16"), dh.PATH_FIELD),           # split forms run on the field
    (1, 0, dict(path="field"), dh.PATH_FIELD),
    (1, 0, dict(max_mg=0), dh.PATH_FIELD),
    (0, 0, dict(max_mg=20), dh.PATH_SPECTRAL),                     # 128x128, two n-tiles
    (1, 0, dict(max_mg=20), dh.PATH_SPECTRAL),
    (4, 0, {}, dh.PATH_SPECTRAL),                                  # 1024x1024 G=30
    (3, 2, {}, dh.PATH_SPECTRAL),                                  # 1024x1024 camera G=15
    (3, 3, {}, dh.PATH_SPECTRAL),                                  # 2048x2048 camera G=20
    (3, 0, dict(max_mg=0), dh.PATH_FIELD),
    (1, 0, dict(ifft_mode=0), dh.PATH_SPECTRAL),                   # IFFT mode 0
    (1, 0, dict(ifft_mode=0, keep_fields=1), dh.PATH_SPECTRAL),    # mode-0 fields by the export
])
def test_path_resolution(idx, cam, kw, path):
    d = dict(dh_synth.config(idx, cam)["params"])
    d.update(kw)
    rc, info = dh.plan_check(d)
    assert rc == dh.SUCCESS and info.path == path


@pytest.mark.parametrize("idx,cam", [(0, 0), (1, 0), (3, 3)])
def test_field_grid_of_both_ifft_modes(idx, cam):
    import oracle
    for mode in (1, 0):
        d = dict(dh_synth.config(idx, cam)["params"], ifft_mode=mode)
        rc, info = dh.plan_check(d)
        g = oracle.geometry(d)
        assert rc == dh.SUCCESS
        assert (info.field_w, info.field_h) == (g["fx"], g["fy"])
        assert info.field_pitch_x == pytest.approx(g["px2"], rel=1e-15)
        assert info.field_pitch_y == pytest.approx(g["py2"], rel=1e-15)
        assert (info.ifft_w, info.ifft_h) == (g["wx"], g["wy"])


def test_int16_conversion_rejects_bad_arguments_without_gpu():
    L = dh.lib()
    assert L.dh_fields_to_int16(None, -1, 4, None, None, None, None) == dh.ERR_INVALIDARGUMENT
    assert L.dh_fields_to_int16(None, 1, 0, None, None, None, None) == dh.ERR_INVALIDARGUMENT
    assert L.dh_fields_to_int16(None, 0, 4, None, None, None, None) == dh.SUCCESS
    assert L.dh_fields_to_int16(None, 2, 4, None, None, None, None) == dh.ERR_NULLPOINTER
    assert L.dh_get_fields16(77, None, None, None, None, None, None, None, None, None, None) == dh.ERR_INVALIDHANDLE


def test_basis_rejects_bad_handles_without_gpu():
    assert dh.lib().dh_set_basis(91, dh.BASIS_LG, 0, 0, None) == dh.ERR_INVALIDHANDLE


@pytest.mark.parametrize("wrap", [False, True])
def test_max_window_radius_matches_oracle(wrap):
    import oracle
    rng = np.random.default_rng(8 + wrap)
    base = dh_synth.config(1)["params"]
    wmax = oracle.w_max_rad(base["pixel_size"], base["wavelength"]) / oracle.DEG
    for _ in range(50):
        t = rng.uniform(-wmax, wmax, size=(2, 2))
        d = dict(base, tilt_deg=t.tolist())
        got = dh.max_window_radius(d, wrap)
        ref = oracle.max_window_radius([tuple(t[0]), tuple(t[1])], wmax, wrap)
        assert got == pytest.approx(ref, abs=1e-12)
    # the paper's worked example: window ~0.719 deg at tilt 1.525 deg on both axes
    assert abs(dh.max_window_radius(dict(base, tilt_deg=[[1.525, 1.525], [1.525, 1.525]])) - 0.719) < 3e-3
    assert dh.lib().dh_max_window_radius(None, 0, None) == dh.ERR_NULLPOINTER


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors of dh_params, dh_plan_info and
    dh_align_report have the header's size and every field at the header's
    offset (a small C program built with gcc against include/dh.h)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"dh_params": dh.Params, "dh_plan_info": dh.PlanInfo, "dh_align_report": dh.AlignReport}
    lines = ['#include "dh.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for name, _ in py._fields_:
            lines.append(f'  printf("{cname} {name} %zu\\n", offsetof({cname}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, name, val = line.split()
            got[(cname, name)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for name, _ in py._fields_:
            assert got[(cname, name)] == getattr(py, name).offset, (cname, name)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """With libdh.so absent the binding raises on first use: there is no
    host-side substitute for any step of the path."""
    monkeypatch.setattr(dh, "_lib", None)
    monkeypatch.setattr(dh, "LIB_PATH", str(tmp_path / "libdh.so"))
    with pytest.raises(RuntimeError, match="missing"):
        dh.lib()
    with pytest.raises(RuntimeError, match="missing"):
        dh.plan_check(_p(0))
    with pytest.raises(RuntimeError, match="missing"):
        dh.max_window_radius(_p(0))


class _FakeDevice:
    def __init__(self, index):
        self.index = index


class _FakeTensor:
    """Duck-typed stand-in for a device tensor (no GPU needed)."""

    def __init__(self, numel, elem=4, floating=True, cuda=True, contiguous=True, device=0):
        self._n, self._e, self._f, self.is_cuda, self._c = numel, elem, floating, cuda, contiguous
        self.device = _FakeDevice(device)
        self.dtype = f"fake{elem * 8}{'f' if floating else 'i'}"

    def data_ptr(self):
        return 0x1000

    def numel(self):
        return self._n

    def element_size(self):
        return self._e

    def is_floating_point(self):
        return self._f

    def is_contiguous(self):
        return self._c


@pytest.mark.parametrize("kw,dtype,msg", [
    (dict(cuda=False), dh.INPUT_F32, "GPU memory"),
    (dict(contiguous=False), dh.INPUT_F32, "contiguous"),
    (dict(elem=8), dh.INPUT_F32, "float32"),                       # float64 frames for an f32 plan
    (dict(elem=4, floating=False), dh.INPUT_F32, "float32"),       # int32 frames
    (dict(elem=4), dh.INPUT_U16, "uint16"),                        # float32 frames for a u16 plan
    (dict(numel=3 * 640 * 512 - 1), dh.INPUT_F32, "frames hold"),  # one pixel short of 3 frames
    (dict(device=1), dh.INPUT_F32, "cuda:1"),
])
def test_binding_rejects_bad_frame_buffers(kw, dtype, msg):
    args = dict(numel=3 * 640 * 512, elem=2 if dtype == dh.INPUT_U16 else 4, floating=dtype == dh.INPUT_F32)
    args.update(kw)
    with pytest.raises(ValueError, match=msg):
        dh._frames_ptr(_FakeTensor(**args), 3, 640 * 512, dtype, 0, "dh_process_batch")
    with pytest.raises(ValueError):
        dh._frames_ptr(None, 3, 640 * 512, dtype, 0, "dh_process_batch")
    with pytest.raises(ValueError):
        dh._frames_ptr(np.zeros(4, np.float32), 1, 4, dtype, 0, "dh_process_batch")


def test_binding_accepts_good_frame_buffers():
    t = _FakeTensor(3 * 640 * 512)
    assert dh._frames_ptr(t, 3, 640 * 512, dh.INPUT_F32, 0, "x") == 0x1000
    t = _FakeTensor(2 * 64, elem=2, floating=False)
    assert dh._frames_ptr(t, 2, 64, dh.INPUT_U16, None, "x") == 0x1000
    assert dh._frames_ptr(0x2000, 10 ** 6, 10 ** 6, dh.INPUT_F32, 0, "x") == 0x2000   # raw address: trusted
