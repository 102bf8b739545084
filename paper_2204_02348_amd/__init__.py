"""Python binding of libdh.so (argument marshalling only).

Every step of the holography path runs in the library's gfx950 kernels; this
module converts arguments and results. It raises if the library is missing:
there is no fallback path.

Device memory and streams come from the caller (e.g. PyTorch tensors and
streams): pass anything with ``data_ptr()`` (or an int address) as frames and
a ``torch.cuda.Stream`` (or an int hipStream_t, or None) as stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdh.so")

SUCCESS = 0
ERR_ERROR = 1
ERR_INVALIDHANDLE = 2
ERR_NULLPOINTER = 3
ERR_INVALIDDIMENSION = 5
ERR_INVALIDPOLARISATION = 6
ERR_INVALIDAXIS = 7
ERR_INVALIDARGUMENT = 8
ERR_MEMORYALLOCATION = 9

INPUT_F32 = 0
INPUT_U16 = 1
PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
PREC_SPLIT_FP16 = 2
METRICS = ["IL", "MDL", "DIAG", "SNRAVG", "DIAGBEST", "DIAGWORST", "SNRBEST", "SNRWORST", "SNRMG"]
GOAL_CAPTURED = -1
BASIS_HG, BASIS_LG, BASIS_CUSTOM = 0, 1, 2
WL_FAST, WL_SLOW = 0, 1
AVG_SEQUENTIAL, AVG_INTERLACED, AVG_SEQUENTIAL_SWEEP = 0, 1, 2
PATH_AUTO = 0
PATH_FIELD = 1
PATH_SPECTRAL = 2

EXPORTS = ["dh_plan_check", "dh_max_window_radius", "dh_plan", "dh_process_batch", "dh_mode_coefs", "dh_get_window",
           "dh_get_fields", "dh_get_fields16", "dh_fields_to_int16", "dh_get_params", "dh_get_plan_info",
           "dh_set_stage_timing", "dh_stage_times", "dh_autoalign", "dh_get_align_report", "dh_set_align_goal",
           "dh_set_pol_lock", "dh_transfer_metrics", "dh_hermitian_eigenvalues",
           "dh_hermitian_eigenvalues_noalloc", "dh_batch_summary",
           "dh_get_field_axes", "dh_set_basis", "dh_set_wavelengths", "dh_set_averaging",
           "dh_serve_create", "dh_serve_info",
           "dh_serve_submit", "dh_serve_progress", "dh_serve_replay", "dh_serve_stats", "dh_serve_destroy",
           "dh_last_error", "dh_destroy"]
ALIGN_FULL, ALIGN_TWEAK, ALIGN_ESTIMATE = 0, 1, 2
ALIGN_TILT, ALIGN_DEFOCUS, ALIGN_WAIST, ALIGN_CENTRE = 1, 2, 4, 8
# launch stages (DH_STAGE_*): row pass; column pass (FFT along y + window,
# then the IFFT along y on the field path or the contraction with the folded
# tables on the spectral path); field pass (field path only); power norm
STAGES = ["row_fft", "column_fft_window", "field_overlap", "power_norm"]


class DhError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with error {code}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("frame_w", C.c_int), ("frame_h", C.c_int), ("pol_count", C.c_int),
        ("fft_w", C.c_int), ("fft_h", C.c_int),
        ("pixel_size", C.c_double), ("wavelength", C.c_double),
        ("beam_centre", (C.c_double * 2) * 2), ("window_radius_deg", C.c_double),
        ("tilt_deg", (C.c_double * 2) * 2), ("defocus", C.c_double * 2), ("waist", C.c_double),
        ("max_mg", C.c_int), ("input_dtype", C.c_int), ("precision", C.c_int),
        ("ifft_mode", C.c_int), ("keep_window", C.c_int), ("keep_fields", C.c_int), ("path", C.c_int),
    ]


class AlignReport(C.Structure):
    _fields_ = [("evaluations", C.c_int), ("sweeps", C.c_int), ("start_goal_db", C.c_double),
                ("goal_db", C.c_double), ("captured", C.c_double), ("snap_tilt_deg", (C.c_double * 2) * 2),
                ("goal", C.c_int), ("metrics", C.c_double * 9), ("snap_centre", (C.c_double * 2) * 2),
                ("snap_waist", C.c_double), ("plane_tilt_deg", (C.c_double * 2) * 2),
                ("snap_defocus", C.c_double * 2)]


class PlanInfo(C.Structure):
    _fields_ = [
        ("fft_w", C.c_int), ("fft_h", C.c_int), ("ifft_w", C.c_int), ("ifft_h", C.c_int),
        ("box_w", C.c_int), ("box_h", C.c_int), ("modes", C.c_int),
        ("x0", C.c_int * 2), ("y0", C.c_int * 2),
        ("ax", C.c_double * 2), ("ay", C.c_double * 2), ("rx", C.c_double), ("ry", C.c_double),
        ("pitch_x", C.c_double), ("pitch_y", C.c_double),
        ("device_bytes", C.c_size_t), ("chunk", C.c_int), ("path", C.c_int),
        ("field_w", C.c_int), ("field_h", C.c_int), ("field_pitch_x", C.c_double), ("field_pitch_y", C.c_double),
        ("generic", C.c_int),
    ]


_lib = None


def lib():
    """The loaded libdh.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_02348_amd.build`")
        L = C.CDLL(LIB_PATH)
        c64p = C.c_void_p
        L.dh_plan_check.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(PlanInfo)]
        L.dh_plan.argtypes = [C.POINTER(Params), C.c_int, C.c_size_t, C.POINTER(C.c_int)]
        L.dh_max_window_radius.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(C.c_double)]
        L.dh_process_batch.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_void_p]
        L.dh_mode_coefs.argtypes = [C.c_int, c64p, C.POINTER(C.c_void_p), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int]
        for f in (L.dh_get_window, L.dh_get_fields):
            f.argtypes = [C.c_int, c64p, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.POINTER(C.c_int),
                          C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.dh_get_params.argtypes = [C.c_int, C.POINTER(Params)]
        L.dh_get_plan_info.argtypes = [C.c_int, C.POINTER(PlanInfo)]
        L.dh_set_stage_timing.argtypes = [C.c_int, C.c_int]
        L.dh_stage_times.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.dh_autoalign.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_uint, C.c_float, C.c_void_p]
        L.dh_get_align_report.argtypes = [C.c_int, C.POINTER(AlignReport)]
        L.dh_serve_create.argtypes = [C.POINTER(C.c_int), C.c_int, C.c_int, C.c_size_t, C.c_int, C.c_int,
                                      C.POINTER(C.c_int)]
        L.dh_serve_info.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_size_t), C.POINTER(C.c_int)]
        L.dh_serve_submit.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        L.dh_serve_progress.argtypes = [C.c_int, C.POINTER(C.c_int)]
        L.dh_serve_replay.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
        L.dh_serve_stats.argtypes = [C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        L.dh_serve_destroy.argtypes = [C.c_int]
        L.dh_transfer_metrics.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.dh_set_align_goal.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.dh_hermitian_eigenvalues.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.dh_hermitian_eigenvalues_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.dh_batch_summary.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.dh_get_field_axes.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.dh_set_pol_lock.argtypes = [C.c_int, C.c_uint]
        L.dh_set_basis.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]
        L.dh_set_wavelengths.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.dh_set_averaging.argtypes = [C.c_int, C.c_int, C.c_int]
        L.dh_get_fields16.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
        L.dh_fields_to_int16.argtypes = [C.c_void_p, C.c_int, C.c_longlong, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        L.dh_last_error.argtypes = [C.c_int]
        L.dh_destroy.argtypes = [C.c_int]
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int
        L.dh_autoalign.restype = C.c_float
        _lib = L
    return _lib


_DTYPES = {"f32": INPUT_F32, "u16": INPUT_U16, INPUT_F32: INPUT_F32, INPUT_U16: INPUT_U16}
_PRECS = {"fp32": PREC_FP32, "split_bf16": PREC_SPLIT_BF16, "split_fp16": PREC_SPLIT_FP16,
          PREC_FP32: PREC_FP32, PREC_SPLIT_BF16: PREC_SPLIT_BF16, PREC_SPLIT_FP16: PREC_SPLIT_FP16}


_PATHS = {"auto": PATH_AUTO, "field": PATH_FIELD, "spectral": PATH_SPECTRAL}


def make_params(d: dict) -> Params:
    """dh_params from a dict with the field names of include/dh.h (the
    recipes' keys); input_dtype 'f32'/'u16', precision 'fp32'/'split_bf16'/
    'split_fp16', path 'auto'/'field'/'spectral' or the numeric codes."""
    p = Params()
    p.frame_w, p.frame_h, p.pol_count = d["frame_w"], d["frame_h"], d["pol_count"]
    p.fft_w, p.fft_h = d["fft_w"], d["fft_h"]
    p.pixel_size, p.wavelength = d["pixel_size"], d["wavelength"]
    for q in range(2):
        for a in range(2):
            p.beam_centre[q][a] = d["beam_centre"][q][a] if q < len(d["beam_centre"]) else 0.0
            p.tilt_deg[q][a] = d["tilt_deg"][q][a] if q < len(d["tilt_deg"]) else 0.0
        p.defocus[q] = d["defocus"][q] if q < len(d["defocus"]) else 0.0
    p.window_radius_deg = d["window_radius_deg"]
    p.waist = d["waist"]
    p.max_mg = d["max_mg"]
    dt, pr = d.get("input_dtype", "f32"), d.get("precision", "fp32")
    p.input_dtype = dt if isinstance(dt, int) else _DTYPES[dt]
    p.precision = pr if isinstance(pr, int) else _PRECS[pr]
    p.ifft_mode = d.get("ifft_mode", 1)
    p.keep_window = int(bool(d.get("keep_window", 0)))
    p.keep_fields = int(bool(d.get("keep_fields", 0)))
    pa = d.get("path", "auto")
    p.path = pa if isinstance(pa, int) else _PATHS[pa]
    return p


def plan_check(d: dict, max_batch: int = 1):
    """(error code, PlanInfo) from the host-only validation; no GPU needed."""
    info = PlanInfo()
    p = make_params(d)
    rc = lib().dh_plan_check(C.byref(p), max_batch, C.byref(info))
    return rc, info


def max_window_radius(d: dict, wrap: bool = False) -> float:
    """dh_max_window_radius: the largest window radius (degrees) for the tilts in d."""
    p = make_params(d)
    r = C.c_double()
    rc = lib().dh_max_window_radius(C.byref(p), int(wrap), C.byref(r))
    if rc != SUCCESS:
        raise DhError(rc, "dh_max_window_radius")
    return r.value


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "cuda_stream"):
        return x.cuda_stream
    raise TypeError(type(x))


def _frames_ptr(x, n_frames: int, frame_elems: int, input_dtype: int, device, what: str) -> int:
    """Device address of `n_frames` frames of `frame_elems` pixels for a call
    into the library. A tensor-like object (``data_ptr``, ``is_cuda``) must be
    on the plan's GPU, contiguous, of the plan's pixel type (4-byte floats for
    f32 plans, 2-byte integers for u16 plans) and hold at least the frames the
    call reads; anything else raises ValueError before the library is called.
    A raw integer address is the caller's responsibility."""
    if x is None:
        raise ValueError(f"{what}: frames is None")
    if isinstance(x, int):
        return x
    if not hasattr(x, "data_ptr"):
        raise ValueError(f"{what}: frames must be a device tensor or an integer device address, not {type(x)}")
    if hasattr(x, "is_cuda"):
        if not x.is_cuda:
            raise ValueError(f"{what}: frames must be in GPU memory (got a host tensor)")
        if device is not None and getattr(x.device, "index", device) != device:
            raise ValueError(f"{what}: frames are on cuda:{x.device.index}, the plan on cuda:{device}")
        if not x.is_contiguous():
            raise ValueError(f"{what}: frames must be contiguous")
        want = 2 if input_dtype == INPUT_U16 else 4
        if x.element_size() != want or (input_dtype == INPUT_F32) != bool(x.is_floating_point()):
            kind = "uint16" if input_dtype == INPUT_U16 else "float32"
            raise ValueError(f"{what}: the plan reads {kind} pixels, frames have dtype {x.dtype}")
        if x.numel() < n_frames * frame_elems:
            raise ValueError(f"{what}: {n_frames} frames of {frame_elems} pixels needed, frames hold {x.numel()}")
    return x.data_ptr()


def _current_device():
    """The current torch device ordinal if torch is loaded and has a GPU, else None."""
    import sys
    torch = sys.modules.get("torch")
    try:
        return torch.cuda.current_device() if torch is not None and torch.cuda.is_available() else None
    except Exception:
        return None


def _stream(s) -> int:
    if s is None:
        return 0
    if isinstance(s, int):
        return s
    return s.cuda_stream


def hermitian_eigenvalues(a, stream=None) -> np.ndarray:
    """Eigenvalues (ascending) of a Hermitian matrix by the library's FP64
    eigenvalue kernel (dh_hermitian_eigenvalues): the eigen step of the MDL
    metric."""
    m = np.asfortranarray(np.asarray(a, dtype=np.complex128))
    n = m.shape[0]
    if m.shape != (n, n):
        raise ValueError("a square matrix is needed")
    w = np.empty(n, dtype=np.float64)
    rc = lib().dh_hermitian_eigenvalues(m.ctypes.data_as(C.c_void_p), n, w.ctypes.data_as(C.c_void_p),
                                        C.c_void_p(_stream(stream)))
    if rc != SUCCESS:
        raise DhError(rc, "dh_hermitian_eigenvalues")
    return w


NOALLOC_EIG_MAX_N = 256          # DH_NOALLOC_EIG_MAX_N


def hermitian_eigenvalues_noalloc(a_dev, n: int, w_dev, stream=None) -> None:
    """dh_hermitian_eigenvalues_noalloc on device buffers (torch tensors or raw
    addresses): a_dev holds the n x n matrix (complex FP64, column-major), w_dev
    receives the n eigenvalues, ascending. No device memory is allocated."""
    rc = lib().dh_hermitian_eigenvalues_noalloc(C.c_void_p(_ptr(a_dev)), int(n), C.c_void_p(_ptr(w_dev)),
                                                C.c_void_p(_stream(stream)))
    if rc != SUCCESS:
        raise DhError(rc, "dh_hermitian_eigenvalues_noalloc")


def fields_to_int16(fields, n_fields: int, field_len: int, re, im, scale, stream=None):
    """dh_fields_to_int16 on device buffers (torch tensors or raw pointers)."""
    rc = lib().dh_fields_to_int16(C.c_void_p(_ptr(fields)), int(n_fields), int(field_len), C.c_void_p(_ptr(re)),
                                  C.c_void_p(_ptr(im)), C.c_void_p(_ptr(scale)), C.c_void_p(_stream(stream)))
    if rc != SUCCESS:
        raise DhError(rc, "dh_fields_to_int16")


class Plan:
    """A dh_plan handle: tables and workspaces resident on the current device."""

    def __init__(self, d: dict, max_batch: int = 1, hbm_budget: int = 0):
        self._p = make_params(d)
        h = C.c_int(-1)
        rc = lib().dh_plan(C.byref(self._p), max_batch, hbm_budget, C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, "dh_plan")
        self.handle = h.value
        self.max_batch = max_batch
        self.device = _current_device()
        self._avg = 1
        self._frame_elems = self._p.frame_w * self._p.frame_h
        info = PlanInfo()
        rc = lib().dh_get_plan_info(self.handle, C.byref(info))
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_plan_info")
        self.info = info

    def _frames(self, frames, batch: int, what: str) -> int:
        n = max(int(batch), 1) * self._avg
        return _frames_ptr(frames, n, self._frame_elems, self._p.input_dtype, self.device, what)

    def process(self, frames, batch: int, stream=None):
        """dh_process_batch: `batch` outputs from batch x (averaging count) frames."""
        ptr = self._frames(frames, batch, "dh_process_batch")
        rc = lib().dh_process_batch(self.handle, C.c_void_p(ptr), batch, C.c_void_p(_stream(stream)))
        if rc != SUCCESS:
            raise DhError(rc, "dh_process_batch")

    def coefs(self, normalised: bool = True) -> np.ndarray:
        """[batch][pol][mode] complex64 on the host (waits for the stream)."""
        b, m, p = C.c_int(), C.c_int(), C.c_int()
        dev = C.c_void_p()
        rc = lib().dh_mode_coefs(self.handle, None, C.byref(dev), C.byref(b), C.byref(m), C.byref(p), int(normalised))
        if rc != SUCCESS:
            raise DhError(rc, "dh_mode_coefs")
        out = np.empty((b.value, p.value, m.value), dtype=np.complex64)
        if m.value:
            rc = lib().dh_mode_coefs(self.handle, out.ctypes.data_as(C.c_void_p), None, None, None, None,
                                     int(normalised))
            if rc != SUCCESS:
                raise DhError(rc, "dh_mode_coefs")
        return out

    def set_wavelengths(self, lambdas, in_order: int = WL_FAST, out_order: int = WL_FAST):
        """Per-frame wavelengths of a sweep (empty: the plan's wavelength only)."""
        lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64).reshape(-1))
        rc = lib().dh_set_wavelengths(self.handle, lam.ctypes.data_as(C.c_void_p) if lam.size else None, lam.size,
                                      int(in_order), int(out_order))
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_wavelengths")

    def set_averaging(self, count: int, mode: int = AVG_SEQUENTIAL):
        rc = lib().dh_set_averaging(self.handle, int(count), int(mode))
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_averaging")
        self._avg = max(int(count), 1)

    def set_basis(self, basis: int, matrix=None):
        """BASIS_HG, BASIS_LG, or BASIS_CUSTOM with `matrix` (modes_out x modes_in complex)."""
        if basis == BASIS_CUSTOM:
            m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex64))
            rc = lib().dh_set_basis(self.handle, basis, m.shape[0], m.shape[1], m.ctypes.data_as(C.c_void_p))
        else:
            rc = lib().dh_set_basis(self.handle, int(basis), 0, 0, None)
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_basis")

    def set_align_goal(self, goal, pol_independent: bool = False, mul_conj_trans: bool = False):
        """Goal of later autoalign calls: GOAL_CAPTURED, a METRICS index or name."""
        g = METRICS.index(goal) if isinstance(goal, str) else int(goal)
        rc = lib().dh_set_align_goal(self.handle, g, int(pol_independent), int(mul_conj_trans))
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_align_goal")

    def set_pol_lock(self, lock: int):
        """Lock pol 1's tilt and/or defocus (ALIGN_TILT | ALIGN_DEFOCUS) to pol 0's in autoalign."""
        rc = lib().dh_set_pol_lock(self.handle, int(lock))
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_pol_lock")

    def transfer_metrics(self, pol_independent: bool = False, mul_conj_trans: bool = False) -> dict:
        """The nine metrics (dB) of the last batch's transfer matrix (dh_transfer_metrics)."""
        out = (C.c_double * len(METRICS))()
        rc = lib().dh_transfer_metrics(self.handle, int(pol_independent), int(mul_conj_trans), out)
        if rc != SUCCESS:
            raise DhError(rc, "dh_transfer_metrics")
        return {k: float(out[i]) for i, k in enumerate(METRICS)}

    def coefs_device_ptr(self, normalised: bool = True) -> int:
        dev = C.c_void_p()
        rc = lib().dh_mode_coefs(self.handle, None, C.byref(dev), None, None, None, int(normalised))
        if rc != SUCCESS:
            raise DhError(rc, "dh_mode_coefs")
        return dev.value or 0

    def _plane(self, fn, what) -> np.ndarray:
        b, p, w, h = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        rc = fn(self.handle, None, None, C.byref(b), C.byref(p), C.byref(w), C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, what)
        out = np.empty((b.value, p.value, h.value, w.value), dtype=np.complex64)
        rc = fn(self.handle, out.ctypes.data_as(C.c_void_p), None, None, None, None, None)
        if rc != SUCCESS:
            raise DhError(rc, what)
        return out

    def window(self) -> np.ndarray:
        return self._plane(lib().dh_get_window, "dh_get_window")

    def fields(self) -> np.ndarray:
        return self._plane(lib().dh_get_fields, "dh_get_fields")

    def fields16(self):
        """(re, im, scale): int16 [batch][pol][h][w] parts and float32 [batch][pol]
        scales of the last batch's fields, field = (re + i im) / scale."""
        b, p, w, h = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        L = lib()
        rc = L.dh_get_fields16(self.handle, None, None, None, None, None, None,
                               C.byref(b), C.byref(p), C.byref(w), C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_fields16")
        re = np.empty((b.value, p.value, h.value, w.value), dtype=np.int16)
        im = np.empty_like(re)
        sc = np.empty((b.value, p.value), dtype=np.float32)
        rc = L.dh_get_fields16(self.handle, re.ctypes.data_as(C.c_void_p), im.ctypes.data_as(C.c_void_p),
                               sc.ctypes.data_as(C.c_void_p), None, None, None, None, None, None, None)
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_fields16")
        return re, im, sc

    def field_axes(self):
        """(x, y): the field grid's axes in metres from the beam centre (dh_get_field_axes)."""
        w, h = C.c_int(), C.c_int()
        rc = lib().dh_get_field_axes(self.handle, None, None, C.byref(w), C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_field_axes")
        x, y = np.empty(w.value), np.empty(h.value)
        rc = lib().dh_get_field_axes(self.handle, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                     None, None)
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_field_axes")
        return x, y

    def batch_summary(self, plane: int, frames=None, batch: int = 0, stream=None):
        """dh_batch_summary: (params [7][pol][batch+1] float64 with MAXABSIDX as
        integers, summed intensity [pol][h][w], x axis, y axis). plane 0: the
        Fourier plane of `batch` frames; plane 1: the last batch's fields."""
        tc, npol, w, h = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        ptr = 0
        if plane == 0:
            ptr = _frames_ptr(frames, max(int(batch), 1), self._frame_elems, self._p.input_dtype, self.device,
                              "dh_batch_summary")
        L = lib()
        rc = L.dh_batch_summary(self.handle, int(plane), C.c_void_p(ptr), int(batch), C.c_void_p(_stream(stream)),
                                None, None, None, None, C.byref(tc), C.byref(npol), C.byref(w), C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, "dh_batch_summary")
        par = np.empty((7, npol.value, tc.value), dtype=np.float32)
        tot = np.empty((npol.value, h.value, w.value), dtype=np.float32)
        x, y = np.empty(w.value), np.empty(h.value)
        rc = L.dh_batch_summary(self.handle, int(plane), C.c_void_p(ptr), int(batch), C.c_void_p(_stream(stream)),
                                par.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p),
                                y.ctypes.data_as(C.c_void_p), tot.ctypes.data_as(C.c_void_p), None, None, None, None)
        if rc != SUCCESS:
            raise DhError(rc, "dh_batch_summary")
        out = par.astype(np.float64)
        out[4] = par[4].view(np.int32)
        return out, tot, x, y

    def set_stage_timing(self, on: bool):
        rc = lib().dh_set_stage_timing(self.handle, int(on))
        if rc != SUCCESS:
            raise DhError(rc, "dh_set_stage_timing")

    def stage_times(self) -> dict:
        """{stage: (ms summed, launches)} since timing was enabled or last read."""
        ms = (C.c_double * 4)()
        n = (C.c_int * 4)()
        rc = lib().dh_stage_times(self.handle, ms, n)
        if rc != SUCCESS:
            raise DhError(rc, "dh_stage_times")
        return {STAGES[k]: (ms[k], n[k]) for k in range(4)}

    def autoalign(self, frames, batch: int, mode: int = ALIGN_FULL,
                  what: int = ALIGN_TILT | ALIGN_DEFOCUS | ALIGN_WAIST, tol: float = 1e-4, stream=None) -> float:
        """Goal in dB after alignment; the plan keeps the aligned parameters."""
        ptr = _frames_ptr(frames, max(int(batch), 1), self._frame_elems, self._p.input_dtype, self.device,
                          "dh_autoalign")
        g = lib().dh_autoalign(self.handle, C.c_void_p(ptr), batch, mode, what, tol,
                               C.c_void_p(_stream(stream)))
        if g == -3.4028234663852886e38:
            raise DhError(self.last_error(), "dh_autoalign")
        return g

    def align_report(self) -> AlignReport:
        r = AlignReport()
        rc = lib().dh_get_align_report(self.handle, C.byref(r))
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_align_report")
        return r

    def params(self) -> dict:
        p = Params()
        rc = lib().dh_get_params(self.handle, C.byref(p))
        if rc != SUCCESS:
            raise DhError(rc, "dh_get_params")
        return {"tilt_deg": [[p.tilt_deg[q][a] for a in range(2)] for q in range(2)],
                "defocus": [p.defocus[0], p.defocus[1]], "waist": p.waist,
                "beam_centre": [[p.beam_centre[q][a] for a in range(2)] for q in range(2)]}

    def last_error(self) -> int:
        return lib().dh_last_error(self.handle)

    def destroy(self):
        if getattr(self, "handle", -1) >= 0:
            lib().dh_destroy(self.handle)
            self.handle = -1

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """dh_serve_*: continuous batching over several camera plans."""

    def __init__(self, plans, max_batch: int = 256, hbm_budget: int = 0, use_graphs: bool = True,
                 normalised: bool = True):
        hs = (C.c_int * len(plans))(*[p.handle for p in plans])
        h = C.c_int(-1)
        rc = lib().dh_serve_create(hs, len(plans), max_batch, hbm_budget, int(use_graphs), int(normalised),
                                   C.byref(h))
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_create")
        self.handle = h.value
        self.plans = list(plans)

    def info(self, camera: int):
        lanes, nbytes, per = C.c_int(), C.c_size_t(), C.c_int()
        rc = lib().dh_serve_info(self.handle, camera, C.byref(lanes), C.byref(nbytes), C.byref(per))
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_info")
        return lanes.value, nbytes.value, per.value

    def replay(self, t_arrival, camera, frame_ptrs, results=None) -> np.ndarray:
        """Real-time replay of a request trace; returns completion times (s).
        results: optional list of complex64 host arrays, one per request."""
        t = np.ascontiguousarray(t_arrival, dtype=np.float64)
        cam = np.ascontiguousarray(camera, dtype=np.int32)
        fp = np.ascontiguousarray(frame_ptrs, dtype=np.uint64)
        n = t.size
        done = np.zeros(n, dtype=np.float64)
        outs = None
        if results is not None:
            outs = np.array([r.ctypes.data for r in results], dtype=np.uint64)
        rc = lib().dh_serve_replay(self.handle, n, t.ctypes.data, cam.ctypes.data, fp.ctypes.data,
                                   outs.ctypes.data if outs is not None else None, done.ctypes.data, None)
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_replay")
        return done

    def submit(self, camera: int, frame, result=None):
        if not 0 <= camera < len(self.plans):
            raise ValueError(f"dh_serve_submit: camera {camera} of {len(self.plans)}")
        pl = self.plans[camera]
        ptr = _frames_ptr(frame, 1, pl._frame_elems, pl._p.input_dtype, pl.device, "dh_serve_submit")
        rc = lib().dh_serve_submit(self.handle, camera, C.c_void_p(ptr),
                                   None if result is None else result.ctypes.data)
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_submit")

    def progress(self) -> int:
        n = C.c_int()
        rc = lib().dh_serve_progress(self.handle, C.byref(n))
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_progress")
        return n.value

    def stats(self):
        b, f = C.c_longlong(), C.c_longlong()
        rc = lib().dh_serve_stats(self.handle, C.byref(b), C.byref(f))
        if rc != SUCCESS:
            raise DhError(rc, "dh_serve_stats")
        return b.value, f.value

    def destroy(self):
        if getattr(self, "handle", -1) >= 0:
            lib().dh_serve_destroy(self.handle)
            self.handle = -1

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
